"""Seeded synthetic problem generators for the split-lasso ADMM hot path.

This module draws inputs only: the sensing matrix H, the measurement vector g,
the true reflectivity u, the block split and the scalars rho and lambda.  It
holds none of the solver's arithmetic.  Both the FP64 oracle and the HIP path
receive the arrays produced here.

Conventions (one fixed draw order per generator, numpy PCG64 seeded):
  * CN(0, s2) means Re and Im are independent N(0, s2/2).
  * H is built in FP64 and rounded once to complex64; that rounded array is
    the problem instance (the oracle upcasts it to complex128).
  * g = H u + w is formed in FP64 from the rounded H and then rounded to
    complex64; w ~ CN(0, sigma2 I) with sigma2 = |Hu|^2 / (m 10^(SNR/10)).
  * lambda = ratio * max|H^H g| is evaluated in FP64 from the rounded H and g,
    so both sides see the same scalar.

The sensing model is the bistatic mm-wave one of the paper's imaging system
(Sec. V, sensing equation g = Hu + w, N_m = N_Tx N_Rx N_f), with the
compressive reflector replaced by one random phase per (Tx, Rx, f) row.
"""

from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

C0 = 299_792_458.0  # speed of light, m/s


@dataclasses.dataclass
class Problem:
    name: str
    H: np.ndarray          # complex64, (m, n), C-contiguous
    g: np.ndarray          # complex64, (m,)
    u_true: np.ndarray     # complex128, (n,)
    Q: int
    P: int
    row_off: np.ndarray | None   # int64 (Q+1,) or None = equal split
    col_off: np.ndarray | None   # int64 (P+1,) or None = equal split
    rho: float
    lam: float
    iters: int

    @property
    def m(self) -> int:
        return self.H.shape[0]

    @property
    def n(self) -> int:
        return self.H.shape[1]


def _lambda_from(H: np.ndarray, g: np.ndarray, ratio: float, rows_per_chunk: int = 512) -> float:
    """ratio * max_n |(H^H g)_n| in FP64, streaming H in row chunks."""
    g128 = g.astype(np.complex128)
    acc = np.zeros(H.shape[1], dtype=np.complex128)
    for r0 in range(0, H.shape[0], rows_per_chunk):
        blk = H[r0:r0 + rows_per_chunk].astype(np.complex128)
        acc += blk.conj().T @ g128[r0:r0 + rows_per_chunk]
    return float(ratio * np.max(np.abs(acc)))


def _noisy(H: np.ndarray, u: np.ndarray, snr_db: float, rng: np.random.Generator) -> np.ndarray:
    nz = np.nonzero(u)[0]
    clean = H[:, nz].astype(np.complex128) @ u[nz]
    m = H.shape[0]
    sigma2 = float(np.vdot(clean, clean).real) / (m * 10.0 ** (snr_db / 10.0))
    w = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * np.sqrt(sigma2 / 2.0)
    return (clean + w).astype(np.complex64)


def iid_problem(m: int = 256, n: int = 4096, nnz: int = 20, snr_db: float = 30.0,
                Q: int = 4, P: int = 1, rho: float = 1.0, lam_ratio: float = 0.05,
                iters: int = 200, seed: int = 0, row_off=None, col_off=None,
                name: str | None = None) -> Problem:
    """iid CN(0, 1/m) sensing matrix with an nnz-sparse unit-modulus target.

    Draw order: Re H, Im H, support (without replacement), phases, Re w, Im w.
    Defaults are the small consensus workload: 256 x 4096, Q=4 row blocks of
    64, P=1, rho=1, lambda = 0.05 max|H^H g|, 200 iterations, seed 0.
    """
    rng = np.random.default_rng(seed)
    s = np.sqrt(1.0 / (2.0 * m))
    Hr = rng.standard_normal((m, n)) * s
    Hi = rng.standard_normal((m, n)) * s
    H = (Hr + 1j * Hi).astype(np.complex64)
    del Hr, Hi
    supp = rng.choice(n, size=nnz, replace=False)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=nnz)
    u = np.zeros(n, dtype=np.complex128)
    u[supp] = np.exp(1j * ph)
    g = _noisy(H, u, snr_db, rng)
    lam = _lambda_from(H, g, lam_ratio)
    return Problem(name or f"iid{m}x{n}_Q{Q}P{P}", np.ascontiguousarray(H), g, u, Q, P,
                   None if row_off is None else np.asarray(row_off, np.int64),
                   None if col_off is None else np.asarray(col_off, np.int64),
                   rho, lam, iters)


def cra_geometry(n_tx: int = 16, n_rx: int = 16, n_f: int = 24,
                 nx: int = 40, ny: int = 40, nz: int = 20,
                 aperture: float = 0.3, f_lo: float = 70e9, f_hi: float = 77e9,
                 spacing: float = 5e-3, z0: float = 0.5, spacing_z: float | None = None):
    """Antenna, frequency and voxel coordinates of the CRA-like imaging model.

    Tx on the x axis, Rx on the y axis (two orthogonal linear arrays at z=0,
    as in the paper's imaging set-up, Sec. VI).  Frequencies uniform in
    [f_lo, f_hi].  Voxel grid centred at (0, 0, z0), `spacing` in x and y and
    `spacing_z` (default: `spacing`) in z; column index
    iz + nz*(iy + ny*ix) (x slowest), so equal column blocks are x slabs.
    Row index rx + n_rx*(tx + n_tx*f) (frequency slowest).
    """
    tx = np.zeros((n_tx, 3))
    tx[:, 0] = np.linspace(-aperture / 2, aperture / 2, n_tx)
    rx = np.zeros((n_rx, 3))
    rx[:, 1] = np.linspace(-aperture / 2, aperture / 2, n_rx)
    freqs = f_lo + (f_hi - f_lo) * np.arange(n_f) / max(n_f - 1, 1)
    xs = (np.arange(nx) - (nx - 1) / 2) * spacing
    ys = (np.arange(ny) - (ny - 1) / 2) * spacing
    zs = z0 + (np.arange(nz) - (nz - 1) / 2) * (spacing if spacing_z is None else spacing_z)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    vox = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)  # (nx*ny*nz, 3), x slowest
    return tx, rx, freqs, vox


def cra_matrix(tx, rx, freqs, vox, phi: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Row-normalised bistatic sensing matrix, complex64 (m, n).

    h = exp(-j 2 pi f (|t-r| + |r-s|)/c + j phi_{t,s,f}) / (|t-r| |r-s|),
    built in FP64 one (f, tx) slab at a time, each row scaled to unit 2-norm,
    then rounded to complex64.
    """
    n_tx, n_rx, n_f = len(tx), len(rx), len(freqs)
    n = vox.shape[0]
    m = n_tx * n_rx * n_f
    dt = np.linalg.norm(vox[None, :, :] - tx[:, None, :], axis=2)  # (n_tx, n)
    dr = np.linalg.norm(vox[None, :, :] - rx[:, None, :], axis=2)  # (n_rx, n)
    amp_r = 1.0 / dr
    H = np.empty((m, n), dtype=np.complex64)
    phi = phi.reshape(n_f, n_tx, n_rx)

    def slab(task):
        fi, ti = task
        k = 2.0 * np.pi * freqs[fi] / C0
        theta = -k * (dt[ti][None, :] + dr) + phi[fi, ti][:, None]
        amp = amp_r * (1.0 / dt[ti])[None, :]
        re = amp * np.cos(theta)
        im = amp * np.sin(theta)
        nrm = np.sqrt(np.sum(re * re + im * im, axis=1, keepdims=True))
        r0 = n_rx * (ti + n_tx * fi)
        blk = H[r0:r0 + n_rx]
        blk.real = re / nrm
        blk.imag = im / nrm

    tasks = [(fi, ti) for fi in range(n_f) for ti in range(n_tx)]
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(slab, tasks))
    return H


def _patch_target(rng: np.random.Generator, nx: int, ny: int, nz: int,
                  px: int = 15, py: int = 5, n_patches: int = 2) -> np.ndarray:
    """Unit-reflectivity planar patches (px x py voxels in x, y), non-overlapping."""
    px = min(px, nx)
    py = min(py, ny)
    while True:
        vol = np.zeros((nx, ny, nz), dtype=bool)
        ok = True
        for _ in range(n_patches):
            iz = rng.integers(0, nz)
            ix = rng.integers(0, nx - px + 1)
            iy = rng.integers(0, ny - py + 1)
            sl = vol[ix:ix + px, iy:iy + py, iz]
            if sl.any():
                ok = False
                break
            vol[ix:ix + px, iy:iy + py, iz] = True
        if ok:
            break
    u = np.zeros(nx * ny * nz, dtype=np.complex128)
    u[vol.ravel()] = 1.0
    return u


def cra_problem(n_tx: int = 16, n_rx: int = 16, n_f: int = 24, nx: int = 40, ny: int = 40,
                nz: int = 20, Q: int = 4, P: int = 8, rho: float = 1.0, lam_ratio: float = 0.02,
                snr_db: float = 25.0, iters: int = 300, seed: int = 0, patch=(15, 5),
                row_off=None, col_off=None, name: str | None = None, geometry: dict | None = None) -> Problem:
    """CRA-like imaging problem.  Defaults are the full imaging workload:
    m = 16*16*24 = 6144 measurements, n = 40*40*20 = 32000 voxels, Q=4, P=8,
    rho=1, lambda = 0.02 max|H^H g|, 25 dB SNR, 300 iterations, seed 0.
    `geometry` passes spacing, spacing_z, z0 or aperture to cra_geometry.

    Draw order: phi (m values, row order), patch positions, Re w, Im w.
    """
    rng = np.random.default_rng(seed)
    tx, rx, freqs, vox = cra_geometry(n_tx, n_rx, n_f, nx, ny, nz, **(geometry or {}))
    m = n_tx * n_rx * n_f
    phi = rng.uniform(0.0, 2.0 * np.pi, size=m)
    H = cra_matrix(tx, rx, freqs, vox, phi)
    u = _patch_target(rng, nx, ny, nz, patch[0], patch[1])
    g = _noisy(H, u, snr_db, rng)
    lam = _lambda_from(H, g, lam_ratio)
    return Problem(name or f"cra{m}x{H.shape[1]}_Q{Q}P{P}", H, g, u, Q, P,
                   None if row_off is None else np.asarray(row_off, np.int64),
                   None if col_off is None else np.asarray(col_off, np.int64),
                   rho, lam, iters)


def small_consensus() -> Problem:
    """256 x 4096 iid consensus workload (Q=4, P=1, 200 iterations, seed 0)."""
    return iid_problem(name="iid256x4096_Q4P1")


# The Jacobi sectioning step (every column block uses the other blocks'
# previous estimated data) is unstable on this matrix at small rho: on the
# grid {1, 3, 4, 4.5, 5, 5.5, 6, 8} the iterates diverge for rho <= 4.5, stall
# at rho = 5 and converge from rho = 5.5 on.  rho = 6 keeps a margin.
FULL_IMAGING_RHO = 6.0


FULL_IMAGING_NAME = "cra6144x32000_Q4P8"


def full_imaging_name() -> str:
    return FULL_IMAGING_NAME


def full_imaging(seed: int = 0, rho: float = FULL_IMAGING_RHO) -> Problem:
    """6144 x 32000 CRA-like consensus-and-sectioning workload (Q=4, P=8, 300 it)."""
    return cra_problem(seed=seed, rho=rho, name=FULL_IMAGING_NAME)


# The imaging set-up of the paper's timing table (Sec. VI, parameter and
# timing tables): 12 Tx x 12 Rx x 15 frequencies in 70-77 GHz = 2160
# measurements; 75 x 75 x 4 = 22500 pixels of lambda_c x lambda_c x 5 lambda_c
# (lambda_c = c / 73.5 GHz) centred 86 cm from the arrays; 50 iterations of
# each of the three splittings, consensus 4 x 1, sectioning 1 x 3 and both
# 4 x 3.  The paper's rho = 1e5 belongs to its own scaling of H; with rows of
# unit norm the iterates do not move in 50 iterations at that value, while
# rho = 10 is the smallest of {1, 3, 10, 1e5} at which all three splittings
# converge within them (1 x 3 and 4 x 3 diverge at 1; at 3 the 1 x 3 primal
# residual only halves).
PAPER_TABLE_SPLITS = ((4, 1), (1, 3), (4, 3))
PAPER_TABLE_RHO = 10.0
PAPER_TABLE_ITERS = 50
_LAMBDA_C = C0 / 73.5e9


def paper_table_imaging(Q: int = 4, P: int = 3, seed: int = 0, rho: float = PAPER_TABLE_RHO) -> Problem:
    """2160 x 22500 CRA-like workload of the paper's timing table (one H for all splits of a seed)."""
    return cra_problem(n_tx=12, n_rx=12, n_f=15, nx=75, ny=75, nz=4, Q=Q, P=P, rho=rho,
                       iters=PAPER_TABLE_ITERS, seed=seed, name=f"cra2160x22500_Q{Q}P{P}",
                       geometry=dict(spacing=_LAMBDA_C, spacing_z=5 * _LAMBDA_C, z0=0.86))


# --------------------------------------------------------------------------
# Batched scenes sharing one instrument matrix
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Batch:
    """S scenes measured by one instrument.  H0 (m0 x n, complex64) is the
    phase-free, row-normalised CRA-like matrix; its rows come in tiles of
    `tile_rows` consecutive rows (one frequency each).  Scene s uses the
    tiles `tiles[s]` (increasing) with one unit phase per row, so
    H_s = diag(phases[s]) H0[rows of tiles[s], :]; its Q_s row blocks are cut
    at the tile boundaries `cuts[s]` (tile units, 0 .. len(tiles[s]))."""
    name: str
    H0: np.ndarray
    tile_rows: int
    tiles: list
    cuts: list
    phases: list          # complex64 per scene row
    g: list               # complex64 per scene
    u_true: list          # complex128 per scene
    lam: list
    P: int
    rho: float
    iters: int

    @property
    def S(self) -> int:
        return len(self.tiles)

    def rows(self, s: int) -> np.ndarray:
        t = np.asarray(self.tiles[s])
        return (t[:, None] * self.tile_rows + np.arange(self.tile_rows)[None, :]).ravel()

    def scene_H(self, s: int, H0=None) -> np.ndarray:
        """H_s in complex128 from H0 (or from a given dequantised H0)."""
        base = self.H0 if H0 is None else H0
        return self.phases[s].astype(np.complex128)[:, None] * base[self.rows(s)].astype(np.complex128)

    def row_off(self, s: int) -> np.ndarray:
        return np.asarray(self.cuts[s], np.int64) * self.tile_rows


def batch_scenes(S: int = 64, seed0: int = 1000, n_tx: int = 16, n_rx: int = 16, n_f: int = 24,
                 nx: int = 40, ny: int = 40, nz: int = 20, f_min: int = 12, P: int = 8, rho: float = 6.0,
                 lam_ratio: float = 0.02, snr_db: float = 25.0, iters: int = 300, q_choices=(2, 4, 8),
                 patch=(15, 5), name: str | None = None) -> Batch:
    """Scenes from the CRA-like generator that share the instrument.

    H0: the phase-free (phi = 0), row-normalised matrix of the geometry.  Scene
    s draws from seed seed0 + s, in order: the number of frequencies N_f in
    U{f_min .. n_f}; a sorted random subset of that many frequency tiles;
    Q_s in q_choices (raised if needed so that blocks can stay narrow);
    Q_s - 1 distinct cuts among the N_f - 1 interior tile boundaries, redrawn
    until every row block has fewer rows than a column block has columns (the
    inversion-lemma x-update); one phase per scene row; the target patches;
    the noise.
    lambda_s = lam_ratio * max|H_s^H g_s| in FP64.
    """
    tx, rx, freqs, vox = cra_geometry(n_tx, n_rx, n_f, nx, ny, nz)
    tile_rows = n_tx * n_rx
    H0 = cra_matrix(tx, rx, freqs, vox, np.zeros(tile_rows * n_f))
    m0, n = H0.shape
    # widest row block (in tiles) that stays narrower than the narrowest column block
    max_tiles = max(1, (n // P - 1) // tile_rows)
    tiles, cuts, phases, gs, us = [], [], [], [], []
    W = np.zeros((m0, S), dtype=np.complex128)     # conj(phase) * g at each scene's rows
    for s in range(S):
        rng = np.random.default_rng(seed0 + s)
        nf = int(rng.integers(f_min, n_f + 1))
        t = np.sort(rng.choice(n_f, size=nf, replace=False)).astype(np.int32)
        Q = int(q_choices[rng.integers(0, len(q_choices))])
        Q = max(Q, -(-nf // max_tiles))
        Q = min(Q, nf)
        while True:   # cuts redrawn until every row block is narrower than its column block
            inner = np.sort(rng.choice(np.arange(1, nf), size=Q - 1, replace=False)) if Q > 1 else np.array([], int)
            c = np.concatenate([[0], inner, [nf]]).astype(np.int32)
            if np.max(np.diff(c)) <= max_tiles:
                break
        ph = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=nf * tile_rows)).astype(np.complex64)
        u = _patch_target(rng, nx, ny, nz, patch[0], patch[1])
        rows = (t[:, None] * tile_rows + np.arange(tile_rows)[None, :]).ravel()
        nzc = np.nonzero(u)[0]
        clean = ph.astype(np.complex128) * (H0[np.ix_(rows, nzc)].astype(np.complex128) @ u[nzc])
        m = len(rows)
        sigma2 = float(np.vdot(clean, clean).real) / (m * 10.0 ** (snr_db / 10.0))
        w = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) * np.sqrt(sigma2 / 2.0)
        g = (clean + w).astype(np.complex64)
        W[rows, s] = np.conj(ph.astype(np.complex128)) * g.astype(np.complex128)
        tiles.append(t)
        cuts.append(c)
        phases.append(ph)
        gs.append(g)
        us.append(u)
    # lambda_s = ratio * max_n |(H_s^H g_s)_n| with H_s = diag(phase) H0[rows]:
    # all scenes at once as H0^H W, in FP64, streaming H0 in row chunks
    Z = np.zeros((n, S), dtype=np.complex128)
    for r0 in range(0, m0, 512):
        Z += H0[r0:r0 + 512].astype(np.complex128).conj().T @ W[r0:r0 + 512]
    lams = [float(lam_ratio * np.max(np.abs(Z[:, s]))) for s in range(S)]
    return Batch(name or f"batch{S}_cra{tile_rows * n_f}x{H0.shape[1]}", H0, tile_rows, tiles, cuts, phases, gs,
                 us, lams, P, rho, iters)
