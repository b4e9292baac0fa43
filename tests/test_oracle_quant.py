"""Pins of the reference quantisers: the published format definitions, checked
against torch's own bfloat16 and float8_e4m3fn conversions (library routines
independent of this code) and against hand-worked values."""
import numpy as np
import pytest
import torch

from oracle import quant as QZ


def test_e4m3_table_matches_format_definition():
    t = QZ.E4M3_TABLE
    assert t[0x00] == 0.0 and t[0x01] == 2.0 ** -9 and t[0x07] == 7 * 2.0 ** -9
    assert t[0x08] == 2.0 ** -6 and t[0x38] == 1.0 and t[0x7E] == 448.0
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert t[0xB8] == -1.0
    # against torch's float8_e4m3fn interpretation of every code
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(np.isnan(ref), np.isnan(t))
    ok = ~np.isnan(t)
    np.testing.assert_array_equal(ref[ok], t[ok])


def test_e4m3_encoder_hand_values():
    x = np.array([1.0, 1.0625, 1.1875, 440.0, 448.0, 500.0, -1e9, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10,
                  0.0, -0.0, 2.0 ** -6 - 2.0 ** -12], np.float32)
    want = [0x38, 0x38, 0x3A, 0x7E, 0x7E, 0x7E, 0xFE, 0x01, 0x00, 0x02, 0x00, 0x80, 0x08]
    np.testing.assert_array_equal(QZ.e4m3_codes(x), np.array(want, np.uint8))


def test_e4m3_encoder_matches_torch_in_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.standard_normal(20000),
                        rng.standard_normal(20000) * 1e-3, (QZ.E4M3_TABLE[:0x7E] + QZ.E4M3_TABLE[1:0x7F]) / 2])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(QZ.e4m3_codes(x), ref)


def test_bf16_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(50000) * 10.0 ** rng.integers(-20, 20, 50000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 0.0])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(QZ.bf16_codes(x), ref)
    np.testing.assert_array_equal(QZ.bf16_values(QZ.bf16_codes(x)),
                                  torch.from_numpy(x).to(torch.bfloat16).float().numpy())


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_dequantised_error_bounds(storage):
    """Relative element error of the stored value: 2^-8 for bf16 (half an
    ulp of an 8-bit significand); for e4m3
    half a mantissa step (2^-4) of the row-scaled value above 2^-6, and
    2^-10 s_r absolute below it."""
    rng = np.random.default_rng(2)
    H = (rng.standard_normal((64, 300)) + 1j * rng.standard_normal((64, 300))).astype(np.complex64)
    H[3] = 0
    D = QZ.dequantise(H, storage)
    H128 = H.astype(np.complex128)
    if storage == "bf16":
        for part in (np.real, np.imag):
            err = np.abs(part(D) - part(H128))
            assert np.all(err <= 2.0 ** -8 * np.abs(part(H128)))
    else:
        s = QZ.fp8_row_scales(H).astype(np.float64)[:, None]
        assert np.all(s[3] == 1.0) and np.all(D[3] == 0)
        for part in (np.real, np.imag):
            y = np.abs(part(H128)) / s
            err = np.abs(part(D) - part(H128)) / s
            bound = np.where(y >= 2.0 ** -6, 2.0 ** -4 * y, 2.0 ** -10) * (1 + 1e-6)
            assert np.all(err <= bound)
