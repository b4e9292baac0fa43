"""GPU parity: the HIP solver (through the C ABI) against the FP64 oracle.

Bar: normalised error |x_gpu - x_oracle| / |x_oracle| <= 1e-5 on the image v
after K iterations for complex64 storage (FP32 arithmetic), on the same
seeded inputs.  Cases span several workgroup tiles, ragged tails (odd block
widths, rows not a multiple of the row tile), uneven block splits and the
three splittings (consensus P=1, sectioning Q=1, combined), plus the
degenerate ones (Q=P=1, zero iterations, lambda above max|H^H g|).  Each
case runs in the form the library picks, with the two-pass kernels of the
inversion-lemma x-update, and (where the n_j x n_j matrices stay small) in
the direct x-update; the oracle takes the inversion lemma for wide blocks and
the direct solve otherwise, the two pinned equal to 1e-12.
"""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import admm as O
from tests._gpu import check_image, gpu_solve, rel, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _oracle(p, iters, **kw):
    return O.solve(p.H, p.g, p.Q, p.P, p.rho, p.lam, iters, p.row_off, p.col_off, **kw)


def _case(name):
    if name == "consensus256x4096":
        return W.small_consensus(), 200
    if name == "combined_uneven":
        return W.iid_problem(m=300, n=2000, nnz=15, Q=3, P=5, rho=10.0, seed=3,
                             row_off=[0, 90, 200, 300], col_off=[0, 333, 800, 1201, 1600, 2000]), 120
    if name == "sectioning":
        return W.iid_problem(m=200, n=1500, nnz=10, Q=1, P=3, rho=10.0, seed=4), 150
    if name == "unsplit":
        return W.iid_problem(m=128, n=1000, nnz=8, Q=1, P=1, rho=1.0, seed=5), 150
    if name == "ragged_consensus":
        return W.iid_problem(m=131, n=1001, nnz=8, Q=3, P=1, rho=1.0, seed=6), 150
    if name == "cra_small":
        return W.cra_problem(n_tx=8, n_rx=8, n_f=12, nx=20, ny=20, nz=10, Q=4, P=4, rho=10.0,
                             patch=(7, 3), iters=100, seed=7), 100
    if name == "many_sections":
        # more sections than the row epilogue keeps in registers (P - 1 > 7);
        # rho large enough for ten Jacobi sections to converge
        return W.iid_problem(m=200, n=3000, nnz=12, Q=2, P=10, rho=40.0, seed=8), 150
    if name == "wide_blocks":
        # 6000-column blocks: longer than one 4096-column chunk of the whole-row
        # product, which streams them in two (the second partial)
        return W.iid_problem(m=128, n=6000, nnz=10, Q=2, P=1, rho=1.0, seed=9), 150
    # Blocks with m_i >= n_j: the GPU keeps the inversion-lemma x-update, the
    # oracle takes the direct solve of (H^H H + rho I) for them.
    if name == "tall_sectioning":      # 300 x 250 blocks
        return W.iid_problem(m=300, n=1000, nnz=10, Q=1, P=4, rho=10.0, seed=21), 150
    if name == "square_blocks":        # 256 x 256
        return W.iid_problem(m=256, n=512, nnz=10, Q=1, P=2, rho=10.0, seed=22), 150
    if name == "mixed_tall":           # 120 x 100 next to wide blocks
        return W.iid_problem(m=240, n=900, nnz=10, Q=2, P=3, rho=10.0, seed=23, col_off=[0, 100, 400, 900]), 150
    if name == "tall_near_limit":      # 480 x 200: just under (1 + sqrt 2) n_j
        return W.iid_problem(m=480, n=1000, nnz=10, Q=1, P=5, rho=10.0, seed=24), 150
    # more than 8 row blocks: up to 32 replicas in registers, beyond that the
    # z-update reads them twice
    # tall enough for the library to pick the direct x-update by itself
    if name == "tall_auto":            # 600 x 100 blocks (sectioning)
        return W.iid_problem(m=600, n=800, nnz=10, Q=1, P=8, rho=10.0, seed=41), 120
    if name == "tall_consensus_auto":  # 500 x 120 blocks (consensus, g' = g)
        return W.iid_problem(m=1000, n=120, nnz=6, Q=2, P=1, rho=1.0, seed=42), 120
    if name == "tall_combined_uneven":   # 3 x 6 uneven blocks, 200-400 x 90-110
        return W.iid_problem(m=900, n=600, nnz=10, Q=3, P=6, rho=10.0, seed=43, row_off=[0, 200, 500, 900],
                             col_off=[0, 90, 200, 300, 410, 500, 600]), 120
    if name == "forty_row_blocks":     # 40 blocks of 30 rows
        return W.iid_problem(m=1200, n=3000, nnz=10, Q=40, P=1, rho=1.0, seed=27), 100
    if name == "many_row_blocks":      # 12 blocks of 40 rows
        return W.iid_problem(m=480, n=2000, nnz=10, Q=12, P=1, rho=1.0, seed=25), 150
    if name == "many_rows_and_sections":   # 10 x 2, ragged rows
        return W.iid_problem(m=501, n=3000, nnz=10, Q=10, P=2, rho=10.0, seed=26), 150
    # degenerate block shapes and weights
    if name == "one_row_blocks":       # m_i = 1: 8 blocks of one row, two sections
        return W.iid_problem(m=8, n=300, nnz=4, Q=8, P=2, rho=10.0, seed=31), 150
    if name == "one_column_blocks":    # n_j = 1: blocks of 2 x 1 (a single column each)
        return W.iid_problem(m=6, n=12, nnz=3, Q=3, P=12, rho=40.0, seed=32), 150
    if name == "lopsided_sections":    # a 64-column section beside a 4096-column one: the row
        # kernel splits each row's sum for 504 slab workgroups (S = 32), so the
        # 8 parts of the narrow section leave most of its threads' runs empty
        return W.iid_problem(m=256, n=4160, nnz=10, Q=4, P=2, rho=10.0, seed=34, col_off=[0, 64, 4160]), 150
    if name == "lambda_zero":          # lambda = 0: kappa = 0, the least-squares iteration
        return W.iid_problem(m=200, n=1200, nnz=10, Q=2, P=2, rho=10.0, lam_ratio=0.0, seed=33), 150
    raise KeyError(name)


CASES = ["consensus256x4096", "combined_uneven", "sectioning", "unsplit", "ragged_consensus",
         "cra_small", "many_sections", "wide_blocks", "tall_sectioning", "square_blocks", "mixed_tall",
         "tall_near_limit", "many_row_blocks", "many_rows_and_sections", "forty_row_blocks",
         "one_row_blocks", "one_column_blocks", "lambda_zero", "tall_auto", "tall_consensus_auto",
         "tall_combined_uneven", "lopsided_sections"]
# the direct x-update on every case but the one with 40 row blocks of 3000
# columns (40 FP64 3000 x 3000 setup matrices) and the one with 4096-column
# sections (four FP64 4096 x 4096 inverses in the oracle)
DIRECT_CASES = [c for c in CASES if c not in ("forty_row_blocks", "lopsided_sections")]
PARITY_RUNS = ([(c, "auto") for c in CASES] + [(c, "two_pass") for c in CASES]
               + [(c, "direct") for c in DIRECT_CASES])


@functools.lru_cache(maxsize=None)
def _reference(name):
    """(problem, K, oracle result) of a named case, computed once per session."""
    p, K = _case(name)
    return p, K, _oracle(p, K)


@pytest.mark.parametrize("name,path", PARITY_RUNS)
def test_image_matches_oracle(torch_gpu, name, path):
    p, K, (v_ref, hist_ref, st_ref) = _reference(name)
    print(f"case {name} ({path}) m={p.m} n={p.n} Q={p.Q} P={p.P} K={K}", flush=True)
    xup = {"auto": "auto", "two_pass": "lemma", "direct": "direct"}[path]
    plan, g, (v, hist) = gpu_solve(torch_gpu, p, K, history=True, two_pass=(path == "two_pass"), xupdate=xup)
    info = plan.info()
    if path == "two_pass":
        assert info["single_pass"] == 0 and info["direct"] == 0
    if path == "direct":
        assert info["direct"] == 1 and info["single_pass"] == 0
    if name.startswith("tall_") and name.endswith(("_auto", "_uneven")):
        assert path == "two_pass" or info["direct"] == 1
    v = v.cpu().numpy()
    err, emax, nd = check_image(v, v_ref, st_ref.s, p.lam / (p.Q * p.rho))
    print(f"  single pass {info['single_pass']}, direct {info['direct']}: rel err {err:.3e}, "
          f"max element err {emax:.3e}, zero pattern on {nd} entries", flush=True)
    hist = hist.cpu().numpy()
    assert hist.shape == hist_ref.shape
    # residual histories: relative agreement where they are well above rounding
    for col in (0, 1):
        ref = hist_ref[:, col]
        big = ref > 1e-6 * ref.max()
        np.testing.assert_allclose(hist[big, col], ref[big], rtol=2e-3)
    # full state (duals, estimated data) after K iterations
    k, vg, sg, ghg = plan.get_state()
    assert k == K
    # duals relative to their size, floored at 1e-3 |u|: with lambda = 0 and
    # more columns than rows every block's data is fitted exactly and the
    # duals converge to 0 (|s| = 2e-9 at K = 150 beside |u| = 1.9), so only
    # FP32 rounding of u is left in them
    s_scale = max(np.linalg.norm(st_ref.s), 1e-3 * np.linalg.norm(st_ref.u))
    assert np.linalg.norm(sg.cpu().numpy() - st_ref.s) <= 10 * TOL * s_scale
    assert rel(ghg.cpu().numpy(), st_ref.ghat) <= 10 * TOL


@pytest.mark.parametrize("name,xupdate", [("combined_uneven", "auto"), ("ragged_consensus", "auto"),
                                          ("cra_small", "auto"), ("gram_patches", "auto"),
                                          ("tall_combined_uneven", "direct"), ("combined_uneven", "direct"),
                                          ("gram_patches_direct", "direct")])
def test_gram_patches_match_oracle(torch_gpu, name, xupdate):
    """The Gram apply in 4 x 4 tile patches (forced; by default only splits
    with thousands of patches use them): single-tile-row blocks, partial edge
    patches and several full patches per block; in the direct form the
    z-update adds the patch pieces itself."""
    import paper_1811_05571_amd as A
    if name == "gram_patches":
        # 600-row blocks: 10 tile rows, patches (R, C) for R, C < 3 with a partial last row
        p, K = W.iid_problem(m=1200, n=6000, nnz=20, Q=2, P=2, rho=10.0, seed=12), 80
    elif name == "gram_patches_direct":
        # 2000 x 600 blocks in the direct form: 10 tile rows of A, as above
        p, K = W.iid_problem(m=2000, n=1200, nnz=20, Q=1, P=2, rho=10.0, seed=13), 80
    else:
        p, K = _case(name)
    v_ref, _, st_ref = _oracle(p, K)
    plan = A.Plan(to_device(torch_gpu, p.H), p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, gram_patches=True,
                  xupdate=xupdate)
    assert plan.info()["gram_patches"] > 0
    assert plan.info()["direct"] == (1 if xupdate == "direct" else 0)
    v = plan.solve(to_device(torch_gpu, p.g), K).cpu().numpy()
    err = rel(v, v_ref)
    print(f"case {name} with patches: rel err {err:.3e}", flush=True)
    assert err <= TOL
    k, _, _, ghg = plan.get_state()
    assert rel(ghg.cpu().numpy(), st_ref.ghat) <= 10 * TOL


def test_deterministic(torch_gpu):
    p, K = _case("combined_uneven")
    plan, g, v1 = gpu_solve(torch_gpu, p, 60)
    v2 = plan.solve(g, 60)
    assert torch_gpu.equal(v1, v2), "two runs from the zero state must be bitwise equal"


@pytest.mark.parametrize("name", ["consensus256x4096", "combined_uneven"])
def test_row_sum_split_matches_one_thread_per_row(torch_gpu, monkeypatch, name):
    """The single pass's row kernel adds a column block's workgroup parts of
    H c with S threads per row (S from ADMM_FZR_LOADS, read at setup): a very
    large limit gives S = 1 (one ordered sum per row); the default split
    (S = 32 for the 512 parts of the 256 x 4096 case) reorders only those FP32
    sums, so both iterate to the same image within the parity bar, 1e-5."""
    import paper_1811_05571_amd as A
    p, K = _case(name)
    H, g = to_device(torch_gpu, p.H), to_device(torch_gpu, p.g)
    monkeypatch.setenv("ADMM_FZR_LOADS", "1000000")
    one = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off)
    monkeypatch.delenv("ADMM_FZR_LOADS")
    split = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off)
    assert one.info()["single_pass"] == 1 and split.info()["single_pass"] == 1
    v1, v2 = one.solve(g, K).cpu().numpy(), split.solve(g, K).cpu().numpy()
    err = rel(v1, v2)
    print(f"{name}: S = 1 against the default split: {err:.2e}")
    assert err <= 1e-5


def test_warm_start_continues(torch_gpu):
    p, K = _case("sectioning")
    plan, g, v_full = gpu_solve(torch_gpu, p, 80)
    plan.solve(g, 50)
    v_warm = plan.solve(g, 30, warm=True)
    assert torch_gpu.equal(v_full, v_warm)


def test_state_roundtrip_matches_oracle(torch_gpu):
    """Import the oracle's state at iteration 40, run 30 more on the GPU,
    compare with 70 oracle iterations."""
    p, _ = _case("combined_uneven")
    _, _, st40 = _oracle(p, 40)
    v70, _, _ = _oracle(p, 30, state=st40)
    torch = torch_gpu
    plan, g, _ = gpu_solve(torch, p, 0)
    plan.set_state(40, to_device(torch, st40.v.astype(np.complex64)),
                   to_device(torch, st40.s.astype(np.complex64)),
                   to_device(torch, st40.ghat.astype(np.complex64)))
    v = plan.solve(g, 30, warm=True).cpu().numpy()
    assert rel(v, v70) <= TOL


def test_warm_start_after_record_and_import(torch_gpu):
    """The single pass keeps the forward parts of H c between solves; a state
    import or a recorded solve (two-pass kernels) makes the next warm solve
    recompute them first: all three continuations equal an uninterrupted run."""
    p, _ = _case("combined_uneven")
    torch = torch_gpu
    plan, g, v_full = gpu_solve(torch, p, 70)
    assert plan.info()["single_pass"] == 1
    plan.solve(g, 40)
    k, v40, s40, gh40 = plan.get_state()
    plan.solve_record(g, 5)                   # moves the state with the two-pass kernels
    plan.set_state(k, v40, s40, gh40)
    v_imp = plan.solve(g, 30, warm=True)
    assert rel(v_imp.cpu().numpy(), v_full.cpu().numpy()) <= 1e-6
    plan.solve(g, 40)
    plan.solve(g, 30, warm=True)              # parts kept from the previous solve
    assert torch.equal(plan.get_state()[1], v_full)


@pytest.mark.parametrize("path", ["single_pass", "two_pass", "direct"])
def test_graph_replay_matches_plain_launches(torch_gpu, path):
    """Solves that replay captured graphs of 10 iterations give bitwise the
    iterates of plain launches: several replays in a row, with the program's
    own eager work (state reads, a plain solve on another plan) and
    synchronisations between them, a remainder shorter than a graph, a new
    lambda (captured again) and the tolerance stop (graphs of check_every
    iterations)."""
    import paper_1811_05571_amd as A
    torch = torch_gpu
    p, _ = _case("combined_uneven")
    H, g = to_device(torch, p.H), to_device(torch, p.g)
    tp = path == "two_pass"
    xu = "direct" if path == "direct" else "auto"
    pg = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, two_pass=tp, xupdate=xu)
    pe = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off, two_pass=tp, xupdate=xu)
    assert pg.info()["direct"] == (1 if path == "direct" else 0)
    pg.set_graphs(True)
    pe.set_graphs(False)
    vg, hg = pg.solve(g, 57, history=True)
    ve, he = pe.solve(g, 57, history=True)
    assert torch.equal(vg, ve) and torch.equal(hg, he)
    for rep in range(4):   # warm replays with eager work between them
        vg = pg.solve(g, 20, warm=True)
        torch.cuda.synchronize()
        kg = pg.get_state()
        ve = pe.solve(g, 20, warm=True)
        ke = pe.get_state()
        assert torch.equal(vg, ve), rep
        assert kg[0] == ke[0] and torch.equal(kg[2], ke[2]) and torch.equal(kg[3], ke[3])
    for plan in (pg, pe):
        plan.set_lambda(0.5 * p.lam)
    assert torch.equal(pg.solve(g, 30), pe.solve(g, 30))
    vg = pg.solve(g, 500, tol=1e-3, check_every=7)
    ve = pe.solve(g, 500, tol=1e-3, check_every=7)
    assert pg.iters_done == pe.iters_done and torch.equal(vg, ve)


def test_zero_iterations_gives_zero_image(torch_gpu):
    p, _ = _case("unsplit")
    _, _, v = gpu_solve(torch_gpu, p, 0)
    assert torch_gpu.count_nonzero(v).item() == 0


def test_lambda_above_max_gives_zero(torch_gpu):
    """lambda >= max|H^H g| makes 0 the minimiser; ADMM reaches it exactly
    once the averaged point falls inside the threshold (consensus, unsplit)."""
    p, _ = _case("unsplit")
    lam = 1.01 * O.lambda_max(p.H, p.g)
    plan, g, v = gpu_solve(torch_gpu, p, 300, lam=lam)
    v_ref, _, _ = O.solve(p.H, p.g, 1, 1, p.rho, lam, 300)
    assert np.max(np.abs(v_ref)) == 0.0
    assert torch_gpu.count_nonzero(v).item() == 0


def test_tolerance_stop_matches_oracle(torch_gpu):
    p, _ = _case("consensus256x4096")
    v_ref, hist_ref, _ = _oracle(p, 500, tol=1e-3, check_every=10)
    plan, g, v = gpu_solve(torch_gpu, p, 500, tol=1e-3, check_every=10)
    assert plan.iters_done == len(hist_ref), (plan.iters_done, len(hist_ref))
    assert rel(v.cpu().numpy(), v_ref) <= TOL


@pytest.mark.parametrize("name", ["consensus256x4096", "combined_uneven", "cra_small"])
def test_kkt_matches_oracle(torch_gpu, name):
    p, K = _case(name)
    plan, g, v = gpu_solve(torch_gpu, p, K)
    got = plan.kkt(g, v)
    want = O.kkt_violation(p.H, p.g, v.cpu().numpy().astype(np.complex128), p.lam)
    assert abs(got - want) <= 1e-9 + 1e-7 * abs(want), (got, want)


def test_nonfinite_g_is_reported(torch_gpu):
    import paper_1811_05571_amd as A
    p, _ = _case("unsplit")
    gbad = p.g.copy()
    gbad[3] = np.nan
    torch = torch_gpu
    plan = A.Plan(to_device(torch, p.H), p.Q, p.P, p.rho, p.lam)
    with pytest.raises(A.ADMMError) as ei:
        plan.solve(to_device(torch, gbad), 5)
    assert ei.value.status == "ADMM_ENONFINITE"


def test_nonfinite_H_is_reported(torch_gpu):
    import paper_1811_05571_amd as A
    p, _ = _case("unsplit")
    Hbad = p.H.copy()
    Hbad[1, 2] = np.inf
    with pytest.raises(A.ADMMError) as ei:
        A.Plan(to_device(torch_gpu, Hbad), p.Q, p.P, p.rho, p.lam)
    assert ei.value.status == "ADMM_ENONFINITE"


def test_bad_arguments_rejected(torch_gpu):
    import paper_1811_05571_amd as A
    p, _ = _case("unsplit")
    H = to_device(torch_gpu, p.H)
    for kw in (dict(rho=0.0), dict(rho=float("nan")), dict(lam=-1.0)):
        args = dict(Q=1, P=1, rho=1.0, lam=0.1)
        args.update(kw)
        with pytest.raises(A.ADMMError) as ei:
            A.Plan(H, **args)
        assert ei.value.status == "ADMM_EINVAL"
    plan = A.Plan(H, 1, 1, 1.0, 0.1)
    # NULL g / v_out and negative iteration counts are argument errors
    assert A.lib().admm_solve(plan.handle, None, 1, 0.0, 1, None, None, None, 0, None) == -1
    g = to_device(torch_gpu, p.g)
    v = torch_gpu.empty(p.n, dtype=torch_gpu.complex64, device="cuda")
    assert A.lib().admm_solve(plan.handle, g.data_ptr(), -1, 0.0, 1, v.data_ptr(), None, None, 0, None) == -1
    assert A.lib().admm_solve(plan.handle, g.data_ptr(), 1, 1e-3, 0, v.data_ptr(), None, None, 0, None) == -1


@pytest.mark.parametrize("path", ["single_pass", "two_pass", "direct"])
def test_profile_sampling_counts_and_leaves_results_unchanged(torch_gpu, path):
    """Kernel timing on every 3rd iteration: 9 iterations give 3 timed launches
    per kernel class of the path, and the iterates are bitwise those of an
    untimed solve."""
    import paper_1811_05571_amd as A
    p, _ = _case("combined_uneven")
    plan, g, (v0, _) = gpu_solve(torch_gpu, p, 9, history=True, two_pass=(path == "two_pass"),
                                 xupdate="direct" if path == "direct" else "auto")
    used = {"single_pass": [A.K_FZ_ROWS, A.K_GRAM, A.K_FZ_SLAB],
            "two_pass": [A.K_GEMV_N, A.K_GRAM, A.K_GEMV_H, A.K_ZUPDATE],
            "direct": [A.K_DIRECT_GP, A.K_GEMV_H, A.K_DIRECT_RHS, A.K_GRAM, A.K_ZUPDATE, A.K_GEMV_N]}[path]
    assert plan.info()["single_pass"] == (1 if path == "single_pass" else 0)
    assert plan.info()["direct"] == (1 if path == "direct" else 0)
    plan.profile(3)
    v1 = plan.solve(g, 9)
    counts = {k: plan.profile_read(k)[1] for k in A.KERNEL_NAMES}
    ms = {k: plan.profile_read(k)[0] for k in A.KERNEL_NAMES}
    plan.profile(0)
    assert counts == {k: (3 if k in used else 0) for k in A.KERNEL_NAMES}
    assert all(ms[k] > 0 for k in used)
    assert torch_gpu.equal(v0, v1)
    with pytest.raises(A.ADMMError):
        plan.profile(-1)
