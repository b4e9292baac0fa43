"""Batched multi-scene form: scenes that share one instrument matrix, with
frequency subsets, per-row phase codes and uneven row splits, solved together
(MFMA GEMMs over the shared bf16 H0, hipGraph replay).  Each scene must match
the FP64 oracle run on that scene's stored matrix diag(phase) bf16(H0)[rows]
(arithmetic error only: FP32 bar 1e-5), graph replay must equal plain
launches bit for bit, and the reconstruction NMSE must equal that of the
plain complex64 solve of the same scene."""
import numpy as np
import pytest

import workloads as W
from oracle import admm as O
from oracle import quant as QZ
from tests._gpu import rel, to_device

pytestmark = pytest.mark.gpu


def _batch():
    # 64-row tiles (8 Tx x 8 Rx), 10 frequencies, 3072 voxels, ragged column split
    return W.batch_scenes(S=6, seed0=1000, n_tx=8, n_rx=8, n_f=10, nx=16, ny=16, nz=12, f_min=4, P=4, rho=10.0,
                          patch=(6, 3), iters=60)


COL_OFF = [0, 700, 1500, 2300, 3072]


def _solve(torch, b, K, graph=True, inverse="c64", gram_patches=False):
    import paper_1811_05571_amd as A
    bb = A.Batch(to_device(torch, b.H0), b.tile_rows, b.tiles, b.cuts, b.phases, b.P, b.rho, b.lam, COL_OFF,
                 inverse=inverse, gram_patches=gram_patches)
    g = to_device(torch, np.concatenate(b.g))
    return bb, g, bb.solve(g, K, graph=graph)


@pytest.mark.parametrize("gram_patches", [False, True])
def test_batch_matches_oracle_per_scene(torch_gpu, gram_patches):
    b = _batch()
    K = 60
    bb, g, v = _solve(torch_gpu, b, K, gram_patches=gram_patches)
    assert (bb.info()["gram_patches"] > 0) == gram_patches   # the small batch is below the size threshold
    v = v.cpu().numpy()
    H0q = QZ.dequantise(b.H0, "bf16")
    worst = 0.0
    for s in range(b.S):
        Hs = b.scene_H(s, H0q)
        ref, _, _ = O.solve(Hs, b.g[s], len(b.cuts[s]) - 1, b.P, b.rho, b.lam[s], K, b.row_off(s), COL_OFF)
        e = rel(v[s], ref)
        print(f"scene {s}: tiles {len(b.tiles[s])} Q {len(b.cuts[s]) - 1} rel err vs oracle {e:.2e}")
        worst = max(worst, e)
    print("tuning", bb.tuning(), bb.info())
    assert worst <= 1e-5


def test_batch_tall_blocks_match_oracle(torch_gpu):
    """Eight equal column blocks of 384: scene 1's 576-row block is taller than
    wide and scene 3 (one row block) square; the oracle solves those blocks
    directly, the batch keeps the inversion lemma."""
    import paper_1811_05571_amd as A
    b = _batch()
    b.cuts[3] = np.array([0, len(b.tiles[3])], dtype=np.int32)
    P, K = 8, 60
    bb = A.Batch(to_device(torch_gpu, b.H0), b.tile_rows, b.tiles, b.cuts, b.phases, P, b.rho, b.lam)
    v = bb.solve(to_device(torch_gpu, np.concatenate(b.g)), K).cpu().numpy()
    H0q = QZ.dequantise(b.H0, "bf16")
    tall = 0
    worst = 0.0
    for s in range(b.S):
        Hs = b.scene_H(s, H0q)
        tall += int(np.diff(b.row_off(s)).max() >= 384)
        ref, _, _ = O.solve(Hs, b.g[s], len(b.cuts[s]) - 1, P, b.rho, b.lam[s], K, b.row_off(s), None)
        worst = max(worst, rel(v[s], ref))
    print(f"tall-block batch: {tall} scenes with blocks of m_i >= n_j, worst rel err {worst:.2e}", flush=True)
    assert tall >= 2 and worst <= 1e-5


def test_batch_graph_equals_plain_launches(torch_gpu):
    b = _batch()
    bb, g, v1 = _solve(torch_gpu, b, 20, graph=True)
    v2 = bb.solve(g, 20, graph=False)
    v3 = bb.solve(g, 20, graph=True)
    assert torch_gpu.equal(v1, v2) and torch_gpu.equal(v1, v3)


def test_batch_nmse_equals_plain_form(torch_gpu):
    """Reconstruction quality of the batched bf16-instrument solve against the
    plain complex64 solve of each scene (same iterations)."""
    import paper_1811_05571_amd as A
    b = _batch()
    K = 60
    bb, g, v = _solve(torch_gpu, b, K)
    v = v.cpu().numpy()
    for s in range(b.S):
        Hs = b.scene_H(s).astype(np.complex64)
        plan = A.Plan(to_device(torch_gpu, Hs), len(b.cuts[s]) - 1, b.P, b.rho, b.lam[s], b.row_off(s), COL_OFF)
        vp = plan.solve(to_device(torch_gpu, b.g[s]), K).cpu().numpy()
        nb = np.linalg.norm(v[s] - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2
        npl = np.linalg.norm(vp - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2
        print(f"scene {s}: NMSE batched {nb:.5f} plain {npl:.5f}")
        assert abs(nb - npl) <= 0.01 * npl + 1e-4


def test_batch_inverse_bf16(torch_gpu):
    """The bfloat16 copy of the scene inverses: every scene within 2^-8 of the
    oracle on its stored matrix (the inverse entries are perturbed by at most
    2^-9 relative), reconstruction error unchanged to 1 %, graph replay equal
    to plain launches."""
    b = _batch()
    K = 60
    bb, g, v = _solve(torch_gpu, b, K, inverse="bf16")
    v2 = bb.solve(g, K, graph=False)
    assert torch_gpu.equal(v, v2)
    v = v.cpu().numpy()
    _, _, v32 = _solve(torch_gpu, b, K)
    v32 = v32.cpu().numpy()
    H0q = QZ.dequantise(b.H0, "bf16")
    for s in range(b.S):
        ref, _, _ = O.solve(b.scene_H(s, H0q), b.g[s], len(b.cuts[s]) - 1, b.P, b.rho, b.lam[s], K, b.row_off(s),
                            COL_OFF)
        e = rel(v[s], ref)
        n16 = np.linalg.norm(v[s] - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2
        n32 = np.linalg.norm(v32[s] - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2
        print(f"scene {s}: bf16 inverse vs oracle {e:.2e}, NMSE {n32:.5f} / {n16:.5f}")
        assert e <= 2.0 ** -8
        assert abs(n16 - n32) <= 1e-2 * n32


def test_batch_rejects_bad_tables(torch_gpu):
    import paper_1811_05571_amd as A
    b = _batch()
    H0 = to_device(torch_gpu, b.H0)
    bad_tiles = [np.array([3, 2, 5], np.int32)] + b.tiles[1:]
    with pytest.raises(A.ADMMError) as ei:
        A.Batch(H0, b.tile_rows, bad_tiles, b.cuts, b.phases, b.P, b.rho, b.lam, COL_OFF)
    assert ei.value.status == "ADMM_EINVAL"
