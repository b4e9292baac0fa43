"""MI355X split-lasso ADMM (consensus / sectioning / both) -- Python binding.

Thin ctypes layer over libadmm.so (C ABI in include/admm.h).  PyTorch is used
only to allocate device memory (H, g, outputs and the workspace) and to hand
the current HIP stream to the library; every step of the solver runs in the
library's HIP kernels.  There is no fallback: if libadmm.so is missing or no
GPU is present the calls raise.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadmm.so")

ADMM_OK = 0
STATUS = {
    -1: "ADMM_EINVAL", -2: "ADMM_EWORKSPACE", -3: "ADMM_EHIP", -4: "ADMM_ENOTPD",
    -5: "ADMM_ENONFINITE", -6: "ADMM_ESTATE", -7: "ADMM_EUNSUPPORTED",
}
STORAGE = {"c64": 0, "bf16": 1, "fp8": 2}
INVERSE = {"c64": 0, "bf16": 16}   # ADMM_INVERSE_BF16: apply a bfloat16 copy of the block inverses
GRAM_PATCHES = 32                   # ADMM_GRAM_PATCHES: always apply the inverses in 4 x 4 tile patches
TWO_PASS = 64                       # ADMM_TWO_PASS: iterate with the two-pass kernels
XUPDATE = {"auto": 0, "lemma": 128, "direct": 256}   # ADMM_XUPDATE_LEMMA / ADMM_XUPDATE_DIRECT
K_GEMV_N, K_GRAM, K_GEMV_H, K_ZUPDATE, K_FZ_ROWS, K_FZ_SLAB, K_DIRECT_GP, K_DIRECT_RHS = range(8)
KERNEL_NAMES = {K_GEMV_N: "k_gemv_n", K_GRAM: "k_gram", K_GEMV_H: "k_gemv_h", K_ZUPDATE: "k_zupdate",
                K_FZ_ROWS: "k_fz_rows", K_FZ_SLAB: "k_fz_slab", K_DIRECT_GP: "k_dgp", K_DIRECT_RHS: "k_dbsum"}

# (name, restype, argtypes) for every symbol of include/admm.h
_c = ctypes
_vp, _i64, _int, _dbl, _sz = _c.c_void_p, _c.c_int64, _c.c_int, _c.c_double, _c.c_size_t
SIGNATURES = [
    ("admm_version", _int, []),
    ("admm_strerror", _c.c_char_p, [_int]),
    ("admm_last_error", _c.c_char_p, []),
    ("admm_workspace_bytes", _int, [_i64, _i64, _int, _vp, _int, _vp, _int, _c.POINTER(_sz)]),
    ("admm_split_cost", _int, [_i64, _i64, _int, _vp, _int, _vp, _int, _c.POINTER(_dbl)]),
    ("admm_model_coefficients", _int, [_c.POINTER(_dbl)]),
    ("admm_calibrate", _int, [_vp, _vp, _i64, _i64, _int, _vp, _sz, _vp, _c.POINTER(_dbl)]),
    ("admm_choose_split", _int, [_i64, _i64, _int, _int, _dbl, _vp, _c.POINTER(_int), _c.POINTER(_int),
                                 _c.POINTER(_dbl)]),
    ("admm_shortlist", _int, [_i64, _i64, _int, _int, _dbl, _vp, _int, _vp, _vp, _vp, _c.POINTER(_int),
                              _c.POINTER(_sz)]),
    ("admm_choose_split_measure", _int, [_vp, _vp, _i64, _i64, _int, _int, _dbl, _vp, _int, _vp, _sz, _vp,
                                         _c.POINTER(_int), _c.POINTER(_int), _c.POINTER(_dbl)]),
    ("admm_setup", _int, [_c.POINTER(_vp), _vp, _i64, _i64, _int, _vp, _int, _vp, _dbl, _dbl, _int,
                          _vp, _sz, _vp]),
    ("admm_set_lambda", _int, [_vp, _dbl]),
    ("admm_set_graphs", _int, [_vp, _int]),
    ("admm_solve", _int, [_vp, _vp, _int, _dbl, _int, _vp, _c.POINTER(_int), _vp, _int, _vp]),
    ("admm_tape_bytes", _int, [_vp, _int, _int, _c.POINTER(_sz)]),
    ("admm_solve_record", _int, [_vp, _vp, _int, _int, _vp, _sz, _vp, _vp]),
    ("admm_backward", _int, [_vp, _vp, _vp, _vp, _vp, _c.POINTER(_dbl), _c.POINTER(_dbl), _vp]),
    ("admm_get_state", _int, [_vp, _vp, _vp, _vp, _c.POINTER(_int), _vp]),
    ("admm_set_state", _int, [_vp, _vp, _vp, _vp, _int, _vp]),
    ("admm_kkt", _int, [_vp, _vp, _vp, _c.POINTER(_dbl), _vp]),
    ("admm_kkt_noalloc", _int, [_vp, _vp, _vp, _c.POINTER(_dbl), _vp]),
    ("admm_hty_absmax", _int, [_vp, _vp, _c.POINTER(_dbl), _vp]),
    ("admm_get_stored_h", _int, [_vp, _vp, _vp, _vp, _vp]),
    ("admm_profile", _int, [_vp, _int]),
    ("admm_profile_read", _int, [_vp, _int, _c.POINTER(_dbl), _c.POINTER(_i64)]),
    ("admm_plan_info", _int, [_vp, _c.POINTER(_i64)]),
    ("admm_destroy", None, [_vp]),
    ("admm_batch_workspace_bytes", _int, [_i64, _i64, _int, _int, _vp, _vp, _vp, _vp, _int, _vp, _int,
                                           _c.POINTER(_sz)]),
    ("admm_batch_setup", _int, [_c.POINTER(_vp), _vp, _i64, _i64, _int, _int, _vp, _vp, _vp, _vp, _vp, _int, _vp,
                                _int, _dbl, _vp, _vp, _sz, _vp]),
    ("admm_batch_solve", _int, [_vp, _vp, _int, _vp, _int, _vp]),
    ("admm_batch_profile", _int, [_vp, _int]),
    ("admm_batch_profile_read", _int, [_vp, _int, _c.POINTER(_dbl), _c.POINTER(_i64)]),
    ("admm_batch_info", _int, [_vp, _c.POINTER(_i64)]),
    ("admm_batch_tuning", _int, [_vp, _c.POINTER(_dbl)]),
    ("admm_batch_destroy", None, [_vp]),
]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libadmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_1811_05571_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class ADMMError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        self.code = code
        self.status = STATUS.get(code, str(code))
        detail = L.admm_last_error().decode()
        super().__init__(f"{where}: {self.status}: {detail}")


def _check(code: int, where: str):
    if code != ADMM_OK:
        raise ADMMError(code, where)


def _offsets(o):
    if o is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(o, dtype=np.int64))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _flags(storage: str, inverse: str, gram_patches: bool, two_pass: bool = False, xupdate: str = "auto") -> int:
    return (STORAGE[storage] | INVERSE[inverse] | (GRAM_PATCHES if gram_patches else 0)
            | (TWO_PASS if two_pass else 0) | XUPDATE[xupdate])


def workspace_bytes(m: int, n: int, Q: int, P: int, row_off=None, col_off=None,
                    storage: str = "c64", inverse: str = "c64", gram_patches: bool = False,
                    two_pass: bool = False, xupdate: str = "auto") -> int:
    ro, rp = _offsets(row_off)
    co, cp = _offsets(col_off)
    out = ctypes.c_size_t(0)
    _check(lib().admm_workspace_bytes(m, n, Q, rp, P, cp, _flags(storage, inverse, gram_patches, two_pass, xupdate),
                                      ctypes.byref(out)), "admm_workspace_bytes")
    return int(out.value)


SPLIT_COST_KEYS = ["exchange_elements", "bytes_per_iteration", "setup_fp64_flops", "inverse_bytes", "h_bytes",
                   "workspace_bytes", "max_block_rows", "max_block_cols", "chunks", "gram_patches", "single_pass",
                   "slab_workgroups", "direct", "slab_load", "slab_threads", "gram_span"]


def split_cost(m: int, n: int, Q: int, P: int, row_off=None, col_off=None, storage: str = "c64",
               inverse: str = "c64", gram_patches: bool = False, two_pass: bool = False,
               xupdate: str = "auto") -> dict:
    ro, rp = _offsets(row_off)
    co, cp = _offsets(col_off)
    out = (ctypes.c_double * 16)()
    _check(lib().admm_split_cost(m, n, Q, rp, P, cp, _flags(storage, inverse, gram_patches, two_pass, xupdate),
                                 out), "admm_split_cost")
    return {k: float(out[i]) for i, k in enumerate(SPLIT_COST_KEYS)}


N_COEF = 10   # coefficients of the timing model (admm_model_coefficients)


def model_coefficients() -> np.ndarray:
    """The built-in coefficients of the split timing model (MI355X fit)."""
    out = (ctypes.c_double * N_COEF)()
    _check(lib().admm_model_coefficients(out), "admm_model_coefficients")
    return np.array(out[:], dtype=np.float64)


def _coef_arg(coef):
    if coef is None:
        return None, None
    arr = (ctypes.c_double * N_COEF)(*[float(x) for x in coef])
    return arr, ctypes.cast(arr, ctypes.c_void_p)


def choose_split(m: int, n: int, iters: int, storage: str = "c64", max_exchange: float = 0.0, coef=None):
    """(Q, P, modelled seconds) of admm_choose_split (coef None: built-in)."""
    q, p, t = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    keep, cp = _coef_arg(coef)
    _check(lib().admm_choose_split(m, n, int(iters), STORAGE[storage], float(max_exchange), cp, ctypes.byref(q),
                                   ctypes.byref(p), ctypes.byref(t)), "admm_choose_split")
    return int(q.value), int(p.value), float(t.value)


def _probe_workspace(torch, H, splits, storage):
    m, n = H.shape
    nb = 0
    for (Q, P, tp) in splits:
        Q, P = min(Q, m), min(P, n)
        nb = max(nb, workspace_bytes(m, n, Q, P, storage=storage, two_pass=tp))
    return torch.empty(nb, dtype=torch.uint8, device=H.device)


CALIBRATION_PROBES = [(4, 4, False), (16, 16, False), (2, 1, False), (32, 32, False), (20, 4, False),
                      (4, 4, True), (8, 2, False)]


def calibrate(H, g, storage: str = "c64", workspace=None) -> np.ndarray:
    """Coefficients of the timing model measured on H's device (admm_calibrate).
    Without a workspace one large enough for every probe is allocated."""
    import torch
    ws = workspace if workspace is not None else _probe_workspace(torch, H, CALIBRATION_PROBES, storage)
    out = (ctypes.c_double * N_COEF)()
    m, n = H.shape
    _check(lib().admm_calibrate(_ptr(H), _ptr(g), m, n, STORAGE[storage], _ptr(ws), ws.numel(),
                                _stream(torch, H.device), out), "admm_calibrate")
    return np.array(out[:], dtype=np.float64)


def shortlist(m: int, n: int, iters: int, k: int, storage: str = "c64", max_exchange: float = 0.0, coef=None):
    """admm_shortlist: the k cheapest candidates [(Q, P, modelled s)] and the
    workspace bytes the largest of them needs."""
    qs, ps, ts = (ctypes.c_int * k)(), (ctypes.c_int * k)(), (ctypes.c_double * k)()
    got, nb = ctypes.c_int(0), ctypes.c_size_t(0)
    keep, cp = _coef_arg(coef)
    _check(lib().admm_shortlist(m, n, int(iters), STORAGE[storage], float(max_exchange), cp, int(k), qs, ps, ts,
                                ctypes.byref(got), ctypes.byref(nb)), "admm_shortlist")
    return [(qs[i], ps[i], ts[i]) for i in range(got.value)], int(nb.value)


def choose_split_measure(H, g, iters: int, storage: str = "c64", max_exchange: float = 0.0, coef=None,
                         shortlist_len: int = 6, workspace=None):
    """(Q, P, measured seconds) of admm_choose_split_measure.  Without a
    workspace one large enough for the shortlist is allocated."""
    import torch
    m, n = H.shape
    if workspace is None:
        _, nb = shortlist(m, n, iters, shortlist_len, storage, max_exchange, coef)
        workspace = torch.empty(nb, dtype=torch.uint8, device=H.device)
    keep, cp = _coef_arg(coef)
    q, p, t = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    _check(lib().admm_choose_split_measure(_ptr(H), _ptr(g), m, n, int(iters), STORAGE[storage],
                                           float(max_exchange), cp, int(shortlist_len), _ptr(workspace),
                                           workspace.numel(), _stream(torch, H.device), ctypes.byref(q),
                                           ctypes.byref(p), ctypes.byref(t)), "admm_choose_split_measure")
    return int(q.value), int(p.value), float(t.value)


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A factored split of H living on one GPU.

    H: torch complex64 CUDA tensor (m, n), row-major contiguous.  The plan
    copies it into its workspace, so H may be freed afterwards.
    """

    def __init__(self, H, Q: int, P: int, rho: float, lam: float, row_off=None, col_off=None,
                 storage: str = "c64", inverse: str = "c64", gram_patches: bool = False, two_pass: bool = False,
                 xupdate: str = "auto"):
        import torch
        if not (H.is_cuda and H.dtype == torch.complex64 and H.dim() == 2 and H.is_contiguous()):
            raise ValueError("H must be a contiguous complex64 CUDA tensor (m, n)")
        self.torch = torch
        self.device = H.device
        self.m, self.n = H.shape
        self.Q, self.P = Q, P
        self.rho, self.lam = float(rho), float(lam)
        self.storage, self.inverse = storage, inverse
        self.row_off, self.col_off = row_off, col_off
        flags = _flags(storage, inverse, gram_patches, two_pass, xupdate)
        nbytes = workspace_bytes(self.m, self.n, Q, P, row_off, col_off, storage, inverse, gram_patches, two_pass,
                                 xupdate)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _, rp = _offsets(row_off)
        _, cp = _offsets(col_off)
        ro_keep, _ = _offsets(row_off)
        co_keep, _ = _offsets(col_off)
        self._keep = (ro_keep, co_keep)
        rp = None if ro_keep is None else ro_keep.ctypes.data_as(ctypes.c_void_p)
        cp = None if co_keep is None else co_keep.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p(0)
        _check(lib().admm_setup(ctypes.byref(h), _ptr(H), self.m, self.n, Q, rp, P, cp, self.rho,
                                self.lam, flags, _ptr(self.workspace), nbytes,
                                _stream(torch, self.device)), "admm_setup")
        self._h = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().admm_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- solver -------------------------------------------------------------
    def set_lambda(self, lam: float):
        _check(lib().admm_set_lambda(self._h, float(lam)), "admm_set_lambda")
        self.lam = float(lam)

    def set_graphs(self, enable: bool):
        """Graph replay of runs of iterations in solve (off by default)."""
        _check(lib().admm_set_graphs(self._h, int(bool(enable))), "admm_set_graphs")

    def solve(self, g, iters: int, tol: float = 0.0, check_every: int = 10, warm: bool = False,
              history: bool = False, out=None):
        """Run `iters` iterations on g (complex64 CUDA, length m); returns v
        (complex64, length n) and, with history=True, a (k, 2) float64 tensor
        of |r_p|^2, |r_d|^2 per iteration."""
        torch = self.torch
        if not (g.is_cuda and g.dtype == torch.complex64 and g.numel() == self.m and g.is_contiguous()):
            raise ValueError("g must be a contiguous complex64 CUDA tensor of length m")
        v = out if out is not None else torch.empty(self.n, dtype=torch.complex64, device=self.device)
        hist = None
        if history:
            # one device buffer kept across solves (a stable pointer lets the
            # library replay its captured graph); the caller gets a copy
            if getattr(self, "_hist", None) is None or self._hist.shape[0] < max(iters, 1):
                self._hist = torch.empty((max(iters, 1), 2), dtype=torch.float64, device=self.device)
            hist = self._hist
        done = ctypes.c_int(0)
        _check(lib().admm_solve(self._h, _ptr(g), int(iters), float(tol), int(check_every), _ptr(v),
                                ctypes.byref(done), None if hist is None else _ptr(hist), int(bool(warm)),
                                _stream(torch, self.device)), "admm_solve")
        self.iters_done = int(done.value)
        if history:
            return v, hist[: self.iters_done].clone()
        return v

    # -- reverse mode -------------------------------------------------------
    def tape_bytes(self, iters: int, interval: int = 10) -> int:
        out = ctypes.c_size_t(0)
        _check(lib().admm_tape_bytes(self._h, int(iters), int(interval), ctypes.byref(out)), "admm_tape_bytes")
        return int(out.value)

    def solve_record(self, g, iters: int, interval: int = 10, tape=None):
        """iters iterations from zero, checkpointing every `interval`; returns
        (v, tape).  The tape is a uint8 device tensor owned by the caller."""
        torch = self.torch
        if not (g.is_cuda and g.dtype == torch.complex64 and g.numel() == self.m and g.is_contiguous()):
            raise ValueError("g must be a contiguous complex64 CUDA tensor of length m")
        nbytes = self.tape_bytes(iters, interval)
        if tape is None or tape.numel() < nbytes:
            tape = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        v = torch.empty(self.n, dtype=torch.complex64, device=self.device)
        _check(lib().admm_solve_record(self._h, _ptr(g), int(iters), int(interval), _ptr(tape), tape.numel(),
                                       _ptr(v), _stream(torch, self.device)), "admm_solve_record")
        return v, tape

    def backward(self, g, grad_v, tape):
        """(dL/dg, dL/dlambda, dL/drho) for the recorded unrolled solve, given
        grad_v = dL/dv^K (convention dL/dRe + j dL/dIm)."""
        torch = self.torch
        grad_v = grad_v.to(torch.complex64).contiguous()
        gg = torch.empty(self.m, dtype=torch.complex64, device=self.device)
        dl = ctypes.c_double(0.0)
        dr = ctypes.c_double(0.0)
        _check(lib().admm_backward(self._h, _ptr(g), _ptr(grad_v), _ptr(tape), _ptr(gg), ctypes.byref(dl),
                                   ctypes.byref(dr), _stream(torch, self.device)), "admm_backward")
        return gg, float(dl.value), float(dr.value)

    def kkt(self, g, v) -> float:
        out = ctypes.c_double(0.0)
        _check(lib().admm_kkt(self._h, _ptr(g), _ptr(v), ctypes.byref(out),
                              _stream(self.torch, self.device)), "admm_kkt")
        return float(out.value)

    def kkt_noalloc(self, g, v) -> float:
        """kkt() with the library's static device scratch instead of the
        plan's workspace (admm_kkt_noalloc)."""
        out = ctypes.c_double(0.0)
        _check(lib().admm_kkt_noalloc(self._h, _ptr(g), _ptr(v), ctypes.byref(out),
                                      _stream(self.torch, self.device)), "admm_kkt_noalloc")
        return float(out.value)

    def hty_absmax(self, g) -> float:
        """max_n |(H^H g)_n| over the stored H, in FP64 (the lasso minimiser is
        zero for lambda at or above it)."""
        out = ctypes.c_double(0.0)
        _check(lib().admm_hty_absmax(self._h, _ptr(g), ctypes.byref(out), _stream(self.torch, self.device)),
               "admm_hty_absmax")
        return float(out.value)

    def get_state(self):
        torch = self.torch
        v = torch.empty(self.n, dtype=torch.complex64, device=self.device)
        s = torch.empty((self.Q, self.n), dtype=torch.complex64, device=self.device)
        ghat = torch.empty((self.P, self.m), dtype=torch.complex64, device=self.device)
        k = ctypes.c_int(0)
        _check(lib().admm_get_state(self._h, _ptr(v), _ptr(s), _ptr(ghat), ctypes.byref(k),
                                    _stream(torch, self.device)), "admm_get_state")
        return int(k.value), v, s, ghat

    def set_state(self, k: int, v, s, ghat):
        _check(lib().admm_set_state(self._h, _ptr(v.contiguous()), _ptr(s.contiguous()),
                                    _ptr(ghat.contiguous()), int(k), _stream(self.torch, self.device)),
               "admm_set_state")

    def stored_h(self):
        """The stored H as dense device tensors: complex64 (C64); uint16 bf16
        codes (re, im) (BF16); uint8 e4m3 codes (re, im) and float32 row scales
        (FP8)."""
        torch = self.torch
        m, n = self.m, self.n
        if self.storage == "c64":
            h = torch.empty((m, n), dtype=torch.complex64, device=self.device)
            _check(lib().admm_get_stored_h(self._h, _ptr(h), None, None, _stream(torch, self.device)),
                   "admm_get_stored_h")
            return h
        dt = torch.int16 if self.storage == "bf16" else torch.uint8
        re = torch.empty((m, n), dtype=dt, device=self.device)
        im = torch.empty((m, n), dtype=dt, device=self.device)
        sc = torch.empty(m, dtype=torch.float32, device=self.device) if self.storage == "fp8" else None
        _check(lib().admm_get_stored_h(self._h, _ptr(re), _ptr(im), None if sc is None else _ptr(sc),
                                       _stream(torch, self.device)), "admm_get_stored_h")
        return re, im, sc

    # -- profiling ----------------------------------------------------------
    def profile(self, every=1):
        """every >= 1: time the kernels of every every-th iteration; 0 / False: off."""
        _check(lib().admm_profile(self._h, int(every)), "admm_profile")

    def profile_read(self, kernel: int):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().admm_profile_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)),
               "admm_profile_read")
        return float(ms.value), int(n.value)

    def info(self) -> dict:
        arr = (ctypes.c_int64 * 16)()
        _check(lib().admm_plan_info(self._h, arr), "admm_plan_info")
        keys = ["m", "n", "Q", "P", "storage", "chunks", "workspace_bytes", "h_bytes", "ginv_bytes",
                "iters_done", "m_pad", "n_pad", "gram_patches", "single_pass", "slab_workgroups", "direct"]
        return {k: int(arr[i]) for i, k in enumerate(keys)}


class Batch:
    """Many scenes sharing one instrument matrix H0 (see include/admm.h).

    H0: complex64 CUDA tensor (m0, n).  tiles, cuts: per-scene integer
    sequences (tile indices; row-block cuts in tile units).  phases: per-scene
    complex64 numpy arrays (one per scene row).  lambdas: per-scene floats."""

    KERNELS = {0: "k_bgemm_n", 1: "k_gram", 2: "k_bgemm_h", 3: "k_bzupdate"}

    def __init__(self, H0, tile_rows: int, tiles, cuts, phases, P: int, rho: float, lambdas, col_off=None,
                 inverse: str = "c64", gram_patches: bool = False):
        import torch
        self.torch = torch
        self.device = H0.device
        self.m0, self.n = H0.shape
        self.tile_rows = int(tile_rows)
        self.S = len(tiles)
        self.P, self.rho = P, float(rho)
        self._tiles = np.ascontiguousarray(np.concatenate([np.asarray(t, np.int32) for t in tiles]))
        self._toff = np.ascontiguousarray(np.cumsum([0] + [len(t) for t in tiles]).astype(np.int64))
        self._cuts = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cuts]))
        self._coff = np.ascontiguousarray(np.cumsum([0] + [len(c) for c in cuts]).astype(np.int64))
        self._lams = np.ascontiguousarray(np.asarray(lambdas, np.float64))
        self._co, cp = _offsets(col_off)
        cp = None if self._co is None else self._co.ctypes.data_as(ctypes.c_void_p)
        self.rows = [len(t) * tile_rows for t in tiles]
        ph = np.concatenate([np.asarray(p_, np.complex64) for p_ in phases])
        self.phases = torch.from_numpy(ph).to(self.device)
        v = ctypes.c_void_p
        args = (self.m0, self.n, int(tile_rows), self.S, self._tiles.ctypes.data_as(v),
                self._toff.ctypes.data_as(v), self._cuts.ctypes.data_as(v), self._coff.ctypes.data_as(v))
        out = ctypes.c_size_t(0)
        flags = INVERSE[inverse] | (GRAM_PATCHES if gram_patches else 0)
        _check(lib().admm_batch_workspace_bytes(*args, P, cp, flags, ctypes.byref(out)), "admm_batch_workspace_bytes")
        self.workspace = torch.empty(int(out.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        _check(lib().admm_batch_setup(ctypes.byref(h), _ptr(H0), *args[:], _ptr(self.phases), P, cp, flags, self.rho,
                                      self._lams.ctypes.data_as(v), _ptr(self.workspace), self.workspace.numel(),
                                      _stream(torch, self.device)), "admm_batch_setup")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().admm_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, g, iters: int, graph: bool = True):
        """g: packed complex64 CUDA tensor of all scenes' rows; returns (S, n)."""
        torch = self.torch
        if not (g.is_cuda and g.dtype == torch.complex64 and g.numel() == sum(self.rows) and g.is_contiguous()):
            raise ValueError("g must be the packed complex64 CUDA measurements of all scenes")
        v = torch.empty((self.S, self.n), dtype=torch.complex64, device=self.device)
        _check(lib().admm_batch_solve(self._h, _ptr(g), int(iters), _ptr(v), int(bool(graph)),
                                      _stream(torch, self.device)), "admm_batch_solve")
        return v

    def profile(self, enable: bool):
        _check(lib().admm_batch_profile(self._h, int(bool(enable))), "admm_batch_profile")

    def profile_read(self, kernel: int):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().admm_batch_profile_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)),
               "admm_batch_profile_read")
        return float(ms.value), int(n.value)

    def info(self) -> dict:
        arr = (ctypes.c_int64 * 16)()
        _check(lib().admm_batch_info(self._h, arr), "admm_batch_info")
        keys = ["m0", "n", "S", "P", "row_blocks", "scene_tiles", "workspace_bytes", "ginv_bytes", "fwd_kchunks",
                "adj_cols_per_wg", "items_n", "items_h", "rows", "fwd_rows_per_wg", "gram_patches"]
        return {k: int(arr[i]) for i, k in enumerate(keys)}

    def tuning(self):
        arr = (ctypes.c_double * 6)()
        _check(lib().admm_batch_tuning(self._h, arr), "admm_batch_tuning")
        # the library's candidate shapes (include/admm.h), rows capped at tile_rows
        rows = [min(r, self.tile_rows) for r in (128, 128, 64)]
        return {"forward_ms": list(arr[:3]), "forward_rows_kchunks": list(zip(rows, (1, 2, 2))),
                "adjoint_ms": list(arr[3:]), "adjoint_cols_per_wg": [64, 128, 256]}


def _unrolled_function():
    import torch

    class UnrolledADMM(torch.autograd.Function):
        """v^K = ADMM(g, lambda, rho) for K iterations from zero, differentiable
        in g, lambda and rho through the library's hand-written adjoint.

        The plan's Gram factors depend on rho, so `rho` must equal plan.rho
        (build a new Plan to change it); lambda is applied with set_lambda."""

        @staticmethod
        def forward(ctx, g, lam, rho, plan, iters, interval):
            if abs(float(rho) - plan.rho) > 1e-12 * max(1.0, plan.rho):
                raise ValueError("rho differs from the plan's rho: build a new Plan")
            plan.set_lambda(float(lam))
            v, tape = plan.solve_record(g.detach().contiguous(), iters, interval)
            ctx.plan, ctx.tape = plan, tape
            ctx.save_for_backward(g)
            return v

        @staticmethod
        def backward(ctx, grad_v):
            (g,) = ctx.saved_tensors
            gg, dl, dr = ctx.plan.backward(g.detach().contiguous(), grad_v, ctx.tape)
            dt = torch.float64
            return gg, torch.tensor(dl, dtype=dt), torch.tensor(dr, dtype=dt), None, None, None

    return UnrolledADMM


def unrolled(g, lam, rho, plan, iters: int, interval: int = 10):
    """Differentiable K-iteration solve (torch.autograd.Function)."""
    global _UNROLLED
    try:
        F = _UNROLLED
    except NameError:
        F = _UNROLLED = _unrolled_function()
    return F.apply(g, lam, rho, plan, iters, interval)
