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


def test_chooser_is_the_argmin_under_the_exchange_limit():
    m, n, K = 2160, 22500, 50
    bw, fl, lat = 6800.0, 45.0, 25.0
    for limit in (0.0, 20000.0, 7000.0):
        q, p, t = A.choose_split(m, n, K, max_exchange=limit, hbm_gbs=bw, fp64_tflops=fl, latency_us=lat)
        best = None
        for Q in CANDIDATES:
            for P in CANDIDATES:
                try:
                    c = A.split_cost(m, n, Q, P)
                except A.ADMMError:
                    continue
                if limit > 0 and c["exchange_elements"] > limit:
                    continue
                tt = c["setup_fp64_flops"] / (fl * 1e12) + K * (c["bytes_per_iteration"] / (bw * 1e9) + lat * 1e-6)
                if best is None or tt < best[2]:
                    best = (Q, P, tt)
        assert (q, p) == best[:2] and t == pytest.approx(best[2], rel=1e-12)
        if limit > 0:
            assert A.split_cost(m, n, q, p)["exchange_elements"] <= limit


def test_chooser_errors():
    # the unsplit problem exchanges nothing: always a candidate, also where its
    # one block is tall (1000 x 300, the direct x-update)
    assert A.choose_split(2160, 22500, 50, max_exchange=1.0)[:2] == (1, 1)
    assert A.choose_split(1000, 300, 50, max_exchange=1.0)[:2] == (1, 1)
    assert A.split_cost(1000, 300, 1, 1)["direct"] == 1
    for kw in (dict(hbm_gbs=0.0), dict(fp64_tflops=-1.0), dict(latency_us=-1.0)):
        with pytest.raises(A.ADMMError) as ei:
            A.choose_split(2160, 22500, 50, **kw)
        assert ei.value.status == "ADMM_EINVAL"
    with pytest.raises(A.ADMMError):
        A.choose_split(2160, 22500, -1)
