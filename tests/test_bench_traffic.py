"""The counter-traffic summary of bench.py (--summarise-traffic): kernels as
rocprofv3 names them (namespace, template arguments, parameter list) map to
the bench's kernel names per storage, the Gram apply's two kernels add up to
one entry, and the copy probe's counts scale the raw KiB (CPU only: the CSV
files are written here)."""
import csv
import json

import bench


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, kib in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_single_pass_kernels_and_gram_pieces(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    probe = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)>(int)"
    seq = [
        (1, probe),
        (2, "void admm::k_fz_rows<admm::FmtC64>(admm::IterArgs, admm::FzArgs, HIP_vector_type<int, 4u> const*)"),
        (3, "void admm::k_gram_tile<false>(admm::IterArgs, HIP_vector_type<int, 4u> const*)"),
        (4, "void admm::k_gram_reduce<false>(admm::IterArgs, HIP_vector_type<int, 4u> const*)"),
        (5, "void admm::k_fz_slab<admm::FmtC64, 1024, 6, true>(admm::IterArgs, admm::FzArgs)"),
    ]
    fetch = {1: 512.0, 2: 10.0, 3: 100.0, 4: 4.0, 5: 1000.0}   # KiB; the probe reads half its MiB here
    write = {1: 1024.0, 2: 1.0, 3: 2.0, 4: 3.0, 5: 20.0}
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(d, n, fetch[d]) for d, n in seq])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(d, n, write[d]) for d, n in seq])
    paths = bench.summarise_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1, "wl", "cmd")
    assert [p.rsplit("/", 1)[-1] for p in paths] == ["traffic_wl_c64.json"]
    rec = json.load(open(paths[0]))
    assert rec["copy_probe"]["fetch_factor"] == 2.0 and rec["copy_probe"]["write_factor"] == 1.0
    k = rec["kernels"]
    assert set(k) == {"k_fz_rows", "k_gram", "k_fz_slab"}
    assert k["k_fz_slab"]["bytes_per_launch"] == (2 * 1000 + 20) * 1024
    assert k["k_fz_rows"]["bytes_per_launch"] == (2 * 10 + 1) * 1024
    # the Gram apply: tile kernel plus its reduction, one entry
    assert k["k_gram"]["bytes_per_launch"] == (2 * 100 + 2 + 2 * 4 + 3) * 1024
    assert sorted(p["kernel"] for p in k["k_gram"]["parts"]) == ["k_gram_reduce<false>", "k_gram_tile<false>"]
    assert rec["kernel_source_sha256_16"] == bench.kernel_source_hash()


def test_shared_kernels_follow_the_storage_of_the_row_product(tmp_path, monkeypatch):
    """A Gram apply dispatched after a bf16 row product counts for bf16."""
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    probe = "at::native::neg_kernel_cuda"
    seq = [
        (1, probe),
        (2, "void admm::k_gemv_nw<admm::FmtBF16, false>(admm::IterArgs, HIP_vector_type<int, 4u> const*)"),
        (3, "void admm::k_gram_tile<false>(admm::IterArgs, HIP_vector_type<int, 4u> const*)"),
        (4, "void admm::k_gemv_h<admm::FmtBF16>(admm::IterArgs, HIP_vector_type<int, 4u> const*)"),
    ]
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(d, n, 1024.0 if d == 1 else 8.0) for d, n in seq])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(d, n, 1024.0 if d == 1 else 1.0) for d, n in seq])
    paths = bench.summarise_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1, "wl", "cmd")
    assert [p.rsplit("/", 1)[-1] for p in paths] == ["traffic_wl_bf16.json"]
    k = json.load(open(paths[0]))["kernels"]
    assert set(k) == {"k_gemv_n", "k_gram", "k_gemv_h"}
    assert all(v["bytes_per_launch"] == 9 * 1024 for v in k.values())
