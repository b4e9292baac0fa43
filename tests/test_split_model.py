"""The split cost model and chooser of the C ABI (host computations, no GPU):
the exchange counts against the paper's tables (Sec. IV and VI), the bytes
per iteration against the benchmark's own algorithmic byte count, and the
chooser against a brute-force search over the same candidates."""
import json
import os

import pytest

import bench
import paper_1811_05571_amd as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CANDIDATES = (1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32)


def test_exchange_counts_match_the_paper():
    gold = json.load(open(os.path.join(GOLDEN, "tab_communications.json")))
    m, n = gold["N_m"], gold["N_p"]
    by = {r["name"]: r for r in gold["printed"]}
    ex = {name: A.split_cost(m, n, r["M"], r["N"])["exchange_elements"] for name, r in by.items()}
    assert ex["consensus"] == by["consensus"]["elements"] == 2 * n
    assert ex["sectioning"] == by["sectioning"]["elements"] == 3 * m
    assert round(100 * (1 - ex["sectioning"] / ex["consensus"]), 1) == by["sectioning"]["reduction_percent"]
    # the combined entry of the example table does not follow the paper's own
    # formula N N_m / M + 2 N_p / N = 3 * 540 + 2 * 7500 (the model keeps the formula)
    assert ex["consensus and sectioning"] == 3 * 540 + 2 * 7500 == 16620 != by["consensus and sectioning"]["elements"]
    assert A.split_cost(m, n, 1, 1)["exchange_elements"] == 0


def test_column_wise_beats_row_wise_below_the_paper_bound():
    """Sec. IV: dividing by columns exchanges less than by rows iff N N_m < 2 N_p."""
    m, n = 2160, 22500
    rows = A.split_cost(m, n, 4, 1)["exchange_elements"]
    for P in (2, 10, 20, 21, 24):
        cols = A.split_cost(m, n, 1, P)["exchange_elements"]
        assert (cols < rows) == (P * m < 2 * n)


@pytest.mark.parametrize("path", ["auto", "two_pass", "direct"])
@pytest.mark.parametrize("Q,P", [(4, 8), (1, 8), (4, 1), (2, 3), (1, 32)])
def test_bytes_per_iteration_match_the_benchmark_count(Q, P, path):
    m, n = 6144, 32000
    xup = {"auto": "auto", "two_pass": "lemma", "direct": "direct"}[path]
    c = A.split_cost(m, n, Q, P, two_pass=(path == "two_pass"), xupdate=xup)
    direct = c["direct"] == 1
    algo = bench.algorithmic_bytes(bench.block_geometry(m, n, Q, P, direct), P, Q, int(c["chunks"]), "c64", "c64",
                                   c["gram_patches"] > 0, int(c["slab_workgroups"]))
    assert direct == (path == "direct" or (path == "auto" and (Q, P) == (1, 32)))
    assert c["single_pass"] == (1 if path == "auto" and not direct else 0)
    assert c["bytes_per_iteration"] == bench.iteration_bytes(algo, {"single_pass": c["single_pass"],
                                                                    "direct": c["direct"]})
    assert c["max_block_rows"] == -(-m // Q) and c["max_block_cols"] == -(-n // P)


@pytest.mark.parametrize("m,n,Q,P,direct", [
    (6144, 32000, 4, 8, False), (6144, 32000, 1, 8, False),    # single pass: H once + m_i^2 beats 2 H + n_j^2
    (6144, 32000, 1, 16, True), (6144, 32000, 1, 32, True),    # 6144 x 2000 and 6144 x 1000 blocks
    (2160, 22500, 1, 16, False), (2160, 22500, 1, 32, True),   # the paper table's shape
    (1000, 120, 2, 1, True), (256, 4096, 4, 1, False)])
def test_form_choice_streams_fewer_bytes(m, n, Q, P, direct):
    """Unless fixed by a flag, a plan takes the x-update whose iteration
    streams fewer bytes (Sec. III-B: the original inversion for tall blocks):
    the two forms' counts bracket the choice."""
    c = A.split_cost(m, n, Q, P)
    lem = A.split_cost(m, n, Q, P, xupdate="lemma")
    dr = A.split_cost(m, n, Q, P, xupdate="direct")
    assert (c["direct"] == 1) == direct
    assert dr["direct"] == 1 and lem["direct"] == 0
    assert c["bytes_per_iteration"] == min(lem["bytes_per_iteration"], dr["bytes_per_iteration"]) or not direct
    assert (dr["inverse_bytes"] < lem["inverse_bytes"]) == (n // P < m // Q)
    # the Gram matrices are n_j x n_j in the direct form: the FP64 setup flops
    nj, mi = -(-n // P), -(-m // Q)
    assert dr["setup_fp64_flops"] >= 8 * (nj * (nj + 1) / 2 * (m // Q) + nj ** 3) * Q * (n // P // nj or 1) * 0.99 ** 0


def test_form_flags_are_exclusive():
    import ctypes
    out = ctypes.c_size_t(0)
    L = A.lib()
    assert L.admm_workspace_bytes(600, 800, 1, None, 8, None, A.XUPDATE["lemma"] | A.XUPDATE["direct"],
                                  ctypes.byref(out)) == -1
    assert L.admm_workspace_bytes(600, 800, 1, None, 8, None, A.XUPDATE["direct"], ctypes.byref(out)) == 0


def test_setup_flops_closed_form():
    # one 100 x 300 block: 8 (m(m+1)/2 n + m^3) real flops
    c = A.split_cost(100, 300, 1, 1)
    assert c["setup_fp64_flops"] == 8 * (100 * 101 / 2 * 300 + 100 ** 3)


def _model_time(m, n, Q, P, K, coef):
    """The timing model written out from admm_split_cost's features:
    setup = c0 flops + c1 span + c2 steps + c3 blocks + c4, iteration =
    c5 h512 + c6 h1024 + c7 (other bytes) + c8 blocks + c9."""
    c = A.split_cost(m, n, Q, P)
    h = c["h_bytes"]
    hz = h * c["slab_load"] if c["single_pass"] else 0.0
    edge = c["max_block_cols"] if c["direct"] else c["max_block_rows"]
    fs = [c["setup_fp64_flops"], c["gram_span"], -(-int(edge) // 64), Q * P, 1.0]
    fi = [hz if c["slab_threads"] == 512 else 0.0, hz if c["slab_threads"] == 1024 else 0.0,
          c["bytes_per_iteration"] - h if c["single_pass"] else c["bytes_per_iteration"], Q * P, 1.0]
    return sum(a * b for a, b in zip(fs, coef[:5])) + K * sum(a * b for a, b in zip(fi, coef[5:]))


@pytest.mark.parametrize("coef", ["builtin", "scaled"])
def test_chooser_is_the_argmin_under_the_exchange_limit(coef):
    m, n, K = 2160, 22500, 50
    k = A.model_coefficients()
    if coef == "scaled":      # other coefficients: setup 3x dearer, blocks 10x
        k = k * [3, 3, 3, 3, 3, 1, 1, 1, 10, 1]
    for limit in (0.0, 20000.0, 7000.0):
        q, p, t = A.choose_split(m, n, K, max_exchange=limit, coef=None if coef == "builtin" else k)
        best = None
        for Q in CANDIDATES:
            for P in CANDIDATES:
                c = A.split_cost(m, n, Q, P)
                if limit > 0 and c["exchange_elements"] > limit:
                    continue
                tt = _model_time(m, n, Q, P, K, k)
                if best is None or tt < best[2]:
                    best = (Q, P, tt)
        assert (q, p) == best[:2] and t == pytest.approx(best[2], rel=1e-12)
        short, ws = A.shortlist(m, n, K, 5, max_exchange=limit, coef=None if coef == "builtin" else k)
        assert short[0][:2] == (q, p) and [x[2] for x in short] == sorted(x[2] for x in short)
        assert ws == max(A.split_cost(m, n, Q, P)["workspace_bytes"] for Q, P, _ in short)
        if limit > 0:
            assert A.split_cost(m, n, q, p)["exchange_elements"] <= limit


def test_model_features():
    """The features the timing model prices, against their definitions: the
    single pass's wave load factor (6144 x 32000, Q = 4: 16 waves of six
    64-row groups, 96 groups: 1.0; Q = 1 in 2160 rows: 34 groups on 6 waves
    of six, 36 slots) and the Gram build's span (4 x 8: 32 blocks of 24 x 25
    / 2 tiles in rounds of 512 workgroups, 4000 columns in chunks of 32)."""
    c = A.split_cost(6144, 32000, 4, 8)
    assert c["slab_load"] == 1.0 and c["slab_threads"] == 1024
    assert c["gram_span"] == 125 * -(-(32 * 24 * 25 // 2) // 512)
    c = A.split_cost(2160, 22500, 1, 3)
    assert c["slab_threads"] == 512 and c["slab_load"] == pytest.approx(36 / 34)
    c = A.split_cost(2160, 22500, 20, 3)
    assert c["single_pass"] == 0 and c["slab_load"] == 0 and c["slab_threads"] == 0
    assert len(A.model_coefficients()) == 10 and (A.model_coefficients() >= 0).all()


def test_chooser_errors():
    # the unsplit problem exchanges nothing: always a candidate, also where its
    # one block is tall (1000 x 300, the direct x-update)
    assert A.choose_split(2160, 22500, 50, max_exchange=1.0)[:2] == (1, 1)
    assert A.choose_split(1000, 300, 50, max_exchange=1.0)[:2] == (1, 1)
    assert A.split_cost(1000, 300, 1, 1)["direct"] == 1
    k = A.model_coefficients()
    for bad in (-1.0, float("nan"), float("inf")):
        kk = k.copy()
        kk[3] = bad
        with pytest.raises(A.ADMMError) as ei:
            A.choose_split(2160, 22500, 50, coef=kk)
        assert ei.value.status == "ADMM_EINVAL"
    with pytest.raises(A.ADMMError):
        A.shortlist(2160, 22500, 50, 0)
    with pytest.raises(A.ADMMError):
        A.choose_split(2160, 22500, -1)
