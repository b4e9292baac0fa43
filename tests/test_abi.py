"""The C ABI library loads without a GPU and exports every entry point that
include/admm.h declares; host-only argument checks work on the CPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "admm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(admm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_1811_05571_amd as A
    L = A.lib()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(n for n, _, _ in A.SIGNATURES) == names


def test_status_strings():
    import paper_1811_05571_amd as A
    L = A.lib()
    for code, name in A.STATUS.items():
        assert L.admm_strerror(code).decode().startswith(name)
    assert L.admm_strerror(0).decode() == "ADMM_OK"


def test_workspace_sizing_and_argument_errors():
    import paper_1811_05571_amd as A
    small = A.workspace_bytes(256, 4096, 4, 1)
    assert small > 256 * 4096 * 8            # at least the stored H
    big = A.workspace_bytes(6144, 32000, 4, 8)
    assert big > 6144 * 32000 * 8
    # the bfloat16 copy of the packed inverses: 4 bytes per stored entry more
    # (32 blocks of 24 x 25 / 2 tiles of 64 x 64 at full size)
    inv16 = A.workspace_bytes(6144, 32000, 4, 8, inverse="bf16")
    assert inv16 - big >= 32 * (24 * 25 // 2) * 4096 * 4
    L = A.lib()
    out = ctypes.c_size_t(0)
    assert L.admm_workspace_bytes(256, 4096, 4, None, 1, None, 1024, ctypes.byref(out)) == -1   # unknown flag
    assert L.admm_workspace_bytes(256, 4096, 4, None, 1, None, 128 | 256, ctypes.byref(out)) == -1   # both forms
    # ADMM_GRAM_PATCHES (32) is known; it only adds the patch table
    assert L.admm_workspace_bytes(256, 4096, 4, None, 1, None, 32, ctypes.byref(out)) == 0
    assert A.workspace_bytes(300, 2000, 3, 5, [0, 90, 200, 300], [0, 333, 800, 1201, 1600, 2000]) > 0
    bad = [
        dict(m=0, n=10, Q=1, P=1),
        dict(m=10, n=20, Q=0, P=1),
        dict(m=10, n=20, Q=11, P=1),
        dict(m=10, n=20, Q=1, P=21),
        dict(m=10, n=20, Q=2, P=1, row_off=[0, 5, 11]),
        dict(m=10, n=20, Q=2, P=1, row_off=[0, 5, 5]),
        dict(m=10, n=20, Q=1, P=2, col_off=[1, 5, 20]),
    ]
    for kw in bad:
        with pytest.raises(A.ADMMError) as ei:
            A.workspace_bytes(**kw)
        assert ei.value.status == "ADMM_EINVAL", kw
    # every block shape is served: tall blocks with the single pass keep the
    # inversion-lemma x-update up to about m_i = (1 + sqrt 2) n_j, taller
    # ones take the direct x-update and its n_j x n_j inverses
    assert A.split_cost(6144, 32000, 1, 8)["direct"] == 0       # 6144 x 4000
    assert A.split_cost(480, 1000, 1, 5)["direct"] == 0         # 480 x 200
    assert A.split_cost(500, 1000, 1, 5)["direct"] == 0         # 500 x 200 (row stride 256, 8 tiles of 64)
    for m, n, P in ((1000, 1000, 5), (6144, 32000, 32)):        # 1000 x 200 and 6144 x 1000
        c = A.split_cost(m, n, 1, P)
        assert c["direct"] == 1
        assert c["inverse_bytes"] == P * (-(-(n // P) // 64) * (-(-(n // P) // 64) + 1) // 2) * 4096 * 8
        assert A.workspace_bytes(m, n, 1, P) > 0


def test_null_plan_is_rejected():
    import paper_1811_05571_amd as A
    L = A.lib()
    assert L.admm_set_lambda(None, 1.0) == -1
    assert L.admm_solve(None, None, 1, 0.0, 1, None, None, None, 0, None) == -1
    assert L.admm_profile(None, 1) == -1
    assert L.admm_hty_absmax(None, None, None, None) == -1
    L.admm_destroy(None)


def test_batch_workspace_sizing_and_errors():
    import ctypes

    import numpy as np

    import paper_1811_05571_amd as A
    L = A.lib()
    tiles = np.array([0, 2, 3, 1, 2], np.int32)
    toff = np.array([0, 3, 5], np.int64)
    cuts = np.array([0, 1, 3, 0, 2], np.int32)
    coff = np.array([0, 3, 5], np.int64)
    v = ctypes.c_void_p
    out = ctypes.c_size_t(0)
    rc = L.admm_batch_workspace_bytes(256, 4096, 64, 2, tiles.ctypes.data_as(v), toff.ctypes.data_as(v),
                                      cuts.ctypes.data_as(v), coff.ctypes.data_as(v), 2, None, 0, ctypes.byref(out))
    assert rc == 0 and out.value > 256 * 4096 * 4
    plain = out.value
    # the bfloat16 copy of the inverses adds 4 bytes per stored inverse entry
    rc = L.admm_batch_workspace_bytes(256, 4096, 64, 2, tiles.ctypes.data_as(v), toff.ctypes.data_as(v),
                                      cuts.ctypes.data_as(v), coff.ctypes.data_as(v), 2, None, 16, ctypes.byref(out))
    assert rc == 0 and out.value > plain
    assert L.admm_batch_workspace_bytes(256, 4096, 64, 2, tiles.ctypes.data_as(v), toff.ctypes.data_as(v),
                                        cuts.ctypes.data_as(v), coff.ctypes.data_as(v), 2, None, 1,
                                        ctypes.byref(out)) == -1     # unknown flag
    bad = np.array([0, 3, 2, 1, 2], np.int32)        # not increasing
    assert L.admm_batch_workspace_bytes(256, 4096, 64, 2, bad.ctypes.data_as(v), toff.ctypes.data_as(v),
                                        cuts.ctypes.data_as(v), coff.ctypes.data_as(v), 2, None, 0,
                                        ctypes.byref(out)) == -1
    assert L.admm_batch_workspace_bytes(256, 4096, 48, 2, tiles.ctypes.data_as(v), toff.ctypes.data_as(v),
                                        cuts.ctypes.data_as(v), coff.ctypes.data_as(v), 2, None, 0,
                                        ctypes.byref(out)) == -1
