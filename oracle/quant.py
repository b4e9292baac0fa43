"""Reference quantisers for the stored-H precision forms.

TEST INFRASTRUCTURE ONLY (same rule as oracle/admm.py).

Formats, from their published definitions:
  * bfloat16: the upper 16 bits of an IEEE fp32 value after round to nearest,
    ties to even, of the lower 16 bits.
  * OCP fp8 e4m3 ("e4m3fn"): 1 sign bit, 4 exponent bits with bias 7, 3
    mantissa bits, subnormals, no infinities, S.1111.111 = NaN, largest
    finite magnitude 448.  Values are encoded by round to nearest with ties to
    the even code, saturating at 448.
  * Row scaling for fp8: s_r = (max over row r of |Re h|, |Im h|) / 448 in
    fp32 (1 for an all-zero row); the codes are those of Re h / s_r and
    Im h / s_r (fp32 divisions); the stored value is s_r * e4m3(code).

The encoder here searches the table of all finite e4m3 magnitudes for the
nearest value; it shares nothing with the device quantiser.
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- bfloat16
def bf16_codes(x) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_values(codes) -> np.ndarray:
    return (np.asarray(codes, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# ---------------------------------------------------------------- fp8 e4m3
def e4m3_value(code: int) -> float:
    """Value of one e4m3 code (NaN for the two NaN codes)."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** (1 - 7)
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


E4M3_TABLE = np.array([e4m3_value(c) for c in range(256)], dtype=np.float64)
_MAGS = E4M3_TABLE[:0x7F]          # codes 0x00..0x7E: all finite non-negative values, increasing


def e4m3_codes(y) -> np.ndarray:
    """Nearest e4m3 code (ties to the even code), saturating at +-448."""
    y = np.asarray(y, dtype=np.float32)
    a = np.abs(y).astype(np.float64)
    hi = np.clip(np.searchsorted(_MAGS, a, side="left"), 0, len(_MAGS) - 1)
    lo = np.clip(hi - 1, 0, len(_MAGS) - 1)
    dlo = np.abs(a - _MAGS[lo])
    dhi = np.abs(_MAGS[hi] - a)
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    pick = np.where(a >= _MAGS[-1], len(_MAGS) - 1, pick)
    sign = np.signbit(y).astype(np.uint8) << 7
    return (pick.astype(np.uint8) | sign).astype(np.uint8)


def e4m3_values(codes) -> np.ndarray:
    return E4M3_TABLE[np.asarray(codes, dtype=np.uint8)]


def fp8_row_scales(H) -> np.ndarray:
    H = np.asarray(H, dtype=np.complex64)
    mx = np.maximum(np.abs(H.real), np.abs(H.imag)).max(axis=1).astype(np.float32)
    return np.where(mx > 0, mx / np.float32(448.0), np.float32(1.0)).astype(np.float32)


# ---------------------------------------------------------------- stored H
def quantise(H, storage: str):
    """Codes of the stored H: ('bf16') -> (re, im) uint16; ('fp8') -> (re, im, s)."""
    H = np.asarray(H, dtype=np.complex64)
    if storage == "bf16":
        return bf16_codes(H.real), bf16_codes(H.imag)
    if storage == "fp8":
        s = fp8_row_scales(H)
        re = (H.real / s[:, None]).astype(np.float32)
        im = (H.imag / s[:, None]).astype(np.float32)
        return e4m3_codes(re), e4m3_codes(im), s
    raise ValueError(storage)


def dequantise(H, storage: str) -> np.ndarray:
    """The stored H as complex128 (exact: every stored value is representable)."""
    if storage == "c64":
        return np.asarray(H, dtype=np.complex64).astype(np.complex128)
    q = quantise(H, storage)
    if storage == "bf16":
        return bf16_values(q[0]).astype(np.float64) + 1j * bf16_values(q[1]).astype(np.float64)
    s = q[2].astype(np.float64)[:, None]
    return s * e4m3_values(q[0]) + 1j * (s * e4m3_values(q[1]))
