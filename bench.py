"""Throughput of the split-lasso ADMM hot path on one MI355X.

A step is one ADMM iteration of the full CRA-like imaging workload
(6144 x 32000 complex64 H, Q=4 row blocks x P=8 column blocks): local data
and forward block products, Gram apply with the estimated-data update,
adjoint block products, thresholded consensus mean, dual update and the
residual norms.  Inputs are resident in HBM before the timed region; the
one-off setup (FP64 Gram, Cholesky, inverse) is timed and reported apart.

Prints one JSON line:  metric/value (iterations/s), the per-kernel event
timings, a roofline object for the dominant kernel and the FP64 oracle timed
on the host cores on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
PROFILE_EVERY = 10      # kernel events on every 10th iteration of the timed region
PROFILES = os.path.join(ROOT, "profiles")


ITER_SOURCES = ("k_iter.hip", "k_fused.hip", "gemv.h", "hstore.h", "common.h", "plan.h")


def kernel_source_hash() -> str:
    """Hash of the sources the per-iteration kernels are compiled from; a
    counter summary taken on other sources is not used."""
    h = hashlib.sha256()
    for f in ITER_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1811_05571_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


ELEM_BYTES = {"c64": 8, "bf16": 4, "fp8": 2}   # stored bytes per complex element of H


def algorithmic_bytes(geo: dict, P: int, Q: int, KH: int, storage: str = "c64", inverse: str = "c64",
                      patches: bool = False, slab_wgs: int = 0) -> dict:
    """Bytes each kernel must move per launch, from the kernel's definition
    (not from counters).  Vectors are complex64 (8 B); H elements take
    ELEM_BYTES[storage] (+ 4 B per row of fp8 scales); inverse entries 8 B
    (4 B for the bfloat16 copy).  slab_wgs: workgroups of the single-pass
    slab kernel, each of which writes (and the row kernel reads) its part of
    H c for every row."""
    m, n = geo["m"], geo["n"]
    ginv = geo["ginv_packed"]     # complex elements of the packed lower-tile inverses
    # 64-vectors of Gram-apply pieces (written once, read once): one per tile
    # and row or column, or, with 4 x 4 tile patches, one per patch and row or column
    gparts = geo["gram_parts_patch"] if patches else geo["gram_parts"]
    c = 8
    h = m * n * ELEM_BYTES[storage] + (4 * m * P if storage == "fp8" else 0)
    vec_rows = P * m * c          # one row-space vector (all column blocks)
    vec_cols = Q * n * c          # one column-space vector (all replicas)
    gemv_n = h + vec_cols + m * c + (P - 1) * vec_rows * (P > 1) + vec_rows * (2 if P > 1 else 1)
    gram = ginv * (4 if inverse == "bf16" else c) + 2 * gparts * 64 * c + vec_rows * (4 if P > 1 else 3)
    gemv_h = h + vec_rows + KH * vec_cols
    zupd = KH * vec_cols + 2 * vec_cols * 2 + 2 * n * c
    parts = slab_wgs * m * c
    # single pass: H once, y of every column block, c and s read and written,
    # v read and written, the row parts written; the row kernel reads the
    # parts, g and the other sections' estimates, and writes r (and g')
    fz_slab = h + vec_rows + 4 * vec_cols + 2 * n * c + parts
    fz_rows = parts + m * c + (P - 1) * vec_rows * (P > 1) + vec_rows * (2 if P > 1 else 1)
    # direct x-update (geo from block_geometry(..., direct=True)): the row
    # residuals from g and the estimates, one row vector per block; their
    # adjoint product (as k_gemv_h); d = the partials + rho (c - u_prev); the
    # Gram apply to d, its pieces written once; the z-update reads the
    # pieces, u_prev and s, writes s, c and u, reads and writes v; the row
    # product reads H and u and writes ghat
    d_gp = m * c + 2 * vec_rows
    d_rhs = (KH + 3) * vec_cols
    d_gram = ginv * (4 if inverse == "bf16" else c) + gparts * 64 * c + vec_cols
    d_zupd = gparts * 64 * c + 5 * vec_cols + 2 * n * c
    d_gemv_n = h + vec_cols + vec_rows
    return {"k_gemv_n": gemv_n, "k_gram": gram, "k_gemv_h": gemv_h, "k_zupdate": zupd,
            "k_fz_rows": fz_rows, "k_fz_slab": fz_slab,
            "k_dgp": d_gp, "k_dbsum": d_rhs, "k_gram_direct": d_gram, "k_zupdate_direct": d_zupd,
            "k_gemv_n_direct": d_gemv_n}


DIRECT_KERNELS = ("k_dgp", "k_gemv_h", "k_dbsum", "k_gram_direct", "k_zupdate_direct", "k_gemv_n_direct")


def iteration_bytes(algo: dict, info: dict) -> int:
    """Algorithmic bytes of one iteration on the plan's path (single pass:
    row kernel, Gram apply, slab kernel; direct form: its six kernels; else
    the four two-pass kernels)."""
    if info.get("direct"):
        names = DIRECT_KERNELS
    elif info.get("single_pass"):
        names = ("k_fz_rows", "k_gram", "k_fz_slab")
    else:
        names = ("k_gemv_n", "k_gram", "k_gemv_h", "k_zupdate")
    return int(sum(algo[k] for k in names))


def load_traffic(kernel: str, workload: str):
    """Counter-derived HBM bytes per launch, if a summary taken on the current
    kernel source is committed under profiles/."""
    path = os.path.join(PROFILES, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


COPY_PROBE_KERNEL = "neg_kernel"   # torch's elementwise negation: reads and writes N bytes
# per-iteration kernels as named in the counter output -> bench names, per storage
TRACE_NAMES = {
    "c64": {"k_gemv_n<FmtC64>": "k_gemv_n", "k_gemv_nw<FmtC64>": "k_gemv_n", "k_gemv_h<FmtC64>": "k_gemv_h",
            "k_fz_slab<FmtC64>": "k_fz_slab", "k_fz_rows<FmtC64>": "k_fz_rows"},
    "bf16": {"k_gemv_n<FmtBF16>": "k_gemv_n", "k_gemv_nw<FmtBF16>": "k_gemv_n", "k_gemv_h<FmtBF16>": "k_gemv_h"},
    "fp8": {"k_gemv_n<FmtFP8>": "k_gemv_n", "k_gemv_nw<FmtFP8>": "k_gemv_n", "k_gemv_h<FmtFP8>": "k_gemv_h"},
}
SHARED_NAMES = {"k_gram_tile<false>": "k_gram", "k_gram_tile<true>": "k_gram", "k_gram_patch": "k_gram",
                "k_gram_reduce<false>": "k_gram", "k_gram_reduce<true>": "k_gram", "k_zupdate<4>": "k_zupdate"}


def _short_kernel(name: str) -> str:
    """Kernel name without namespace, arguments and template flags after the
    first template argument (k_gemv_n<FmtFP8, true> -> k_gemv_n<FmtFP8>)."""
    n = name.replace("admm::(anonymous namespace)::", "").replace("admm::", "").replace("void ", "")
    n = n.split("(")[0].strip()
    return re.sub(r"<([^,<>]+),[^<>]*>", r"<\1>", n)


def read_counter_csv(path: str, counter: str) -> list:
    """rocprofv3 --pmc csv -> [(dispatch id, short kernel name, KiB)] in dispatch order."""
    import csv
    per = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            key = (int(row["Dispatch_Id"]), _short_kernel(row["Kernel_Name"]))
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    return sorted((d, k, v) for (d, k), v in per.items())


def _by_storage(disp: list) -> dict:
    """{storage: {kernel: [KiB, ...]}}: a kernel shared by the storages counts
    for the storage of the last storage-typed row product dispatched before it."""
    owner = {n: st for st, names in TRACE_NAMES.items() for n in names}
    out, cur = {}, None
    for _, k, v in disp:
        if k in owner:
            cur = owner[k]
        if k in owner or (k in SHARED_NAMES and cur is not None):
            out.setdefault(cur, {}).setdefault(k, []).append(v)
    return out


def summarise_traffic(fetch_csv: str, write_csv: str, probe_mib: int, workload: str, command: str):
    """Writes profiles/traffic_<workload>_<storage>.json from a FETCH_SIZE and
    a WRITE_SIZE counter run, each scaled by what the counter reads for the
    copy probe (probe_mib MiB read and written)."""
    fetch_d = read_counter_csv(fetch_csv, "FETCH_SIZE")
    write_d = read_counter_csv(write_csv, "WRITE_SIZE")
    probe = sorted({k for _, k, _ in fetch_d if COPY_PROBE_KERNEL in k})
    if len(probe) != 1:
        raise SystemExit(f"copy probe kernel not found once in {fetch_csv}: {probe}")
    pk = probe[0]
    kib = probe_mib * 1024.0
    pf = [v for _, k, v in fetch_d if k == pk]
    pw = [v for _, k, v in write_d if k == pk]
    f_fac = kib / float(np.mean(pf))
    w_fac = kib / float(np.mean(pw))
    fetch, write = _by_storage(fetch_d), _by_storage(write_d)
    written = []
    for storage, names in TRACE_NAMES.items():
        fs, ws = fetch.get(storage, {}), write.get(storage, {})
        kern = {}
        for src, dst in list(names.items()) + list(SHARED_NAMES.items()):
            if src not in fs or src not in ws:
                continue
            fb = float(np.mean(fs[src])) * 1024.0 * f_fac
            wb = float(np.mean(ws[src])) * 1024.0 * w_fac
            k = kern.setdefault(dst, {"fetch_bytes": 0.0, "write_bytes": 0.0, "parts": []})
            k["fetch_bytes"] += fb
            k["write_bytes"] += wb
            k["parts"].append({"kernel": src, "dispatches": len(fs[src]), "fetch_kib_raw": float(np.mean(fs[src])),
                               "write_kib_raw": float(np.mean(ws[src]))})
        if not any(n in kern for n in ("k_gemv_n", "k_gemv_h", "k_fz_slab")):
            continue
        for k in kern.values():
            k["bytes_per_launch"] = int(round(k["fetch_bytes"] + k["write_bytes"]))
        rec = {"workload": f"{workload}_{storage}", "kernel_source_sha256_16": kernel_source_hash(),
               "copy_probe": {"kernel": pk, "mib": probe_mib, "fetch_factor": f_fac, "write_factor": w_fac,
                              "fetch_kib_raw": float(np.mean(pf)), "write_kib_raw": float(np.mean(pw))},
               "command": command, "kernels": kern}
        path = os.path.join(PROFILES, f"traffic_{workload}_{storage}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        written.append(path)
    return written


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_BF16", "SQ_VALU_MFMA_BUSY_CYCLES",
                 "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")
SIMDS = 256 * 4   # MI355X: 256 CUs of 4 SIMDs
XCDS = 8          # and 8 XCDs, each with its own GRBM


def summarise_mfma(counter_csv: str, trace_csv: str, command: str, workload: str = "batch64_cra6144x32000"):
    """profiles/mfma_<workload>.md: per batched GEMM kernel, the mean per
    dispatch of the MFMA counters, the MFMA flops they give (MOPS x 512),
    the kernel-trace duration, and the MFMA-busy fraction
    SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x SIMDs): the
    busy cycles are summed over all SIMDs, GRBM_GUI_ACTIVE over the 8 XCDs
    (each counts the kernel's cycles)."""
    import csv
    per = {}
    with open(counter_csv) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            if "k_bgemm" not in name:
                continue
            if row["Counter_Name"] not in MFMA_COUNTERS:
                continue
            key = (_short_kernel(name), int(row["Dispatch_Id"]))
            per.setdefault(key, {}).setdefault(row["Counter_Name"], 0.0)
            per[key][row["Counter_Name"]] += float(row["Counter_Value"])
    dur = {}
    with open(trace_csv) as f:
        for row in csv.DictReader(f):
            if "k_bgemm" not in row["Kernel_Name"]:
                continue
            dur.setdefault(_short_kernel(row["Kernel_Name"]), []).append(
                (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9)
    lines = [f"# MFMA counters: batched complex GEMMs, {workload}", "",
             "One MI355X, ROCm 7.2.  The 64-scene batch (bf16 H0, FP32 vectors split into three bf16 terms:",
             "12 real MFMAs per complex multiply-add) for a few iterations under rocprofv3 counter collection;",
             "durations from the kernel trace of the same run (serialised by the counter collection, so",
             "longer than in the timed bench).", "", "Command (`$REPO` = repository root):", "", "```",
             command, "```", "",
             "| kernel | dispatches | MFMA bf16 instructions | MOPS_BF16 x 512 = MFMA flops | MFMA busy cycles (all SIMDs) | GUI active cycles (sum of 8 XCDs) | MFMA busy fraction | avg trace us | MFMA TFLOP/s |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    kinds = sorted({k for k, _ in per})
    for k in kinds:
        rows = [v for (kk, _), v in per.items() if kk == k]
        mean = {c: float(np.mean([r.get(c, 0.0) for r in rows])) for c in MFMA_COUNTERS}
        flops = mean["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512
        busy = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / max(mean["GRBM_GUI_ACTIVE"] / XCDS * SIMDS, 1.0)
        d = float(np.mean(dur.get(k, [float("nan")])))
        lines.append(f"| `{k}` | {len(rows)} | {mean['SQ_INSTS_VALU_MFMA_BF16']:.4g} | {flops:.4g} | "
                     f"{mean['SQ_VALU_MFMA_BUSY_CYCLES']:.4g} | {mean['GRBM_GUI_ACTIVE']:.4g} | {busy:.3f} | "
                     f"{d * 1e6:.1f} | {flops / d / 1e12:.1f} |")
    path = os.path.join(PROFILES, f"mfma_{workload}.md")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def copy_probe(torch, dev, mib: int, reps: int = 3):
    """A plain elementwise copy of known size (N bytes read, N written) that
    calibrates the memory counters."""
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def attainable_bandwidth(torch, dev, gib: int = 2, reps: int = 5) -> dict:
    """Reference rates of plain streaming on this GPU, best of `reps` timed
    runs each (HIP events on torch's stream): read-only reductions over `gib`
    GiB -- the row sums of a (rows x 4096) float32 view, the same matrix's
    transposed product with a vector, and the flat sum -- and a copy of the
    same size (read and written).  "read_gbs" is the fastest read."""
    n = gib * (1 << 30) // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    X = x.view(-1, 4096)
    Xc = x.view(4096, -1)          # its transpose is a row-major (rows x 4096) operand read once by the gemv
    w = torch.ones(4096, dtype=torch.float32, device=dev)
    out = {}
    reads = (("read_rowsum", lambda: X.sum(1)), ("read_gemv_t", lambda: torch.mv(Xc.t(), w)),
             ("read_flat_sum", lambda: torch.sum(x)))
    for name, fn, nbytes in [(r, f, x.numel() * 4) for r, f in reads] + [("copy", lambda: y.copy_(x),
                                                                          2 * x.numel() * 4)]:
        fn()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        out[f"{name}_gbs"] = round(nbytes / best / 1e9, 1)
    out["read_gbs"] = max(out[f"{r}_gbs"] for r, _ in reads)
    del x, y, X, Xc, w
    torch.cuda.empty_cache()
    out["bytes"] = gib * (1 << 30)
    return out


def _blas_info():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max((d.get("num_threads", 1) for d in info), default=1)
        blas = ",".join(sorted({f"{d.get('internal_api', '?')}" for d in info}))
    except Exception:
        threads, blas = os.cpu_count(), "?"
    return threads, blas


def cpu_baseline(prob, n_iter: int, keep=(), H=None):
    """The FP64 oracle on the host cores in its push-through form (two
    products with each block per iteration, the form a host solver would
    run): setup once, then n_iter iterations timed.  Returns the timing and
    the image after each iteration count in `keep`.  H: the matrix to run on
    (default the workload's complex64 H)."""
    from oracle import admm as O
    threads, blas = _blas_info()
    H = prob.H.astype(np.complex128) if H is None else H
    ro = O.split_offsets(prob.m, prob.Q)
    co = O.split_offsets(prob.n, prob.P)
    t0 = time.perf_counter()
    blocks = O.setup_push_through(H, ro, co, prob.rho)
    t1 = time.perf_counter()
    st = O.State.zeros(prob.m, prob.n, prob.Q, prob.P)
    g = prob.g.astype(np.complex128)
    kept = {}
    for k in range(n_iter):
        st, _, _ = O.step_push_through(g, ro, co, prob.rho, prob.lam, blocks, st)
        if k + 1 in keep:
            kept[k + 1] = st.v.copy()
    t2 = time.perf_counter()
    return {
        "setup_s": t1 - t0, "iter_s": (t2 - t1) / max(n_iter, 1), "iters": n_iter, "threads": threads,
        "blas": blas, "v": st.v, "kept": kept, "cpu": platform.processor() or platform.machine(),
        "affinity": len(os.sched_getaffinity(0)),
    }


CONVERGENCE_CHECKPOINTS = (100, 300, 1000, 3000, 10000)


def convergence_run(plan, g, checkpoints):
    """The solve continued warm from zero through growing iteration counts,
    run back to back (the GPU kept busy): device copies of v and of the last
    residuals at each checkpoint, for convergence_eval."""
    import torch
    pts, done = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in checkpoints:
        v, hist = plan.solve(g, k - done, warm=done > 0, history=True)
        pts.append((k, v, hist[-1].clone()))
        done = k
    torch.cuda.synchronize()
    return pts, time.perf_counter() - t0


def convergence_eval(plan, g, prob, run) -> dict:
    """At each checkpoint of convergence_run: the FP64 KKT violation of v (over
    lambda; zero exactly at the lasso minimiser), the reconstruction NMSE
    against the synthetic truth, the nonzeros and the last iteration's
    |r_p|^2, |r_d|^2.  Where the KKT violation falls while the NMSE levels
    off, the NMSE left is the lasso model's on this geometry, not unfinished
    iterations."""
    pts_dev, t_run = run
    pts = []
    for k, v, last in pts_dev:
        vn = v.cpu().numpy()
        pts.append({"iterations": k, "kkt_violation": plan.kkt(g, v),
                    "nmse_vs_truth": float(np.linalg.norm(vn - prob.u_true) ** 2 / np.linalg.norm(prob.u_true) ** 2),
                    "nonzeros": int(np.count_nonzero(vn)),
                    "final_residuals": [float(x) for x in last.cpu().numpy()]})
        print(f"[bench] convergence: {k} iterations, KKT {pts[-1]['kkt_violation']:.3e}, "
              f"NMSE {pts[-1]['nmse_vs_truth']:.4f}", file=sys.stderr, flush=True)
    return {"checkpoints": pts, "solve_s": round(t_run, 3), "truth_nonzeros": int(np.count_nonzero(prob.u_true)),
            "note": "one solve continued warm through the checkpoints (history on), run back to back before the "
                    "headline's warm-up; KKT violation over lambda"}


def bench_small(args, torch, A, W, dev, reps: int = 5) -> dict:
    """The 256 x 4096 consensus workload (Q = 4 row blocks of 64, P = 1, 200
    iterations): H is 8.4 MB and stays in the caches, so an iteration is
    bound by launches and latency, not HBM (no roofline claim).  Median of
    `reps` 200-iteration solves with plain launches and with graph replay."""
    p = W.small_consensus()
    H, g = torch.from_numpy(p.H).to(dev), torch.from_numpy(p.g).to(dev)
    plan = A.Plan(H, p.Q, p.P, p.rho, p.lam, p.row_off, p.col_off)
    out = {"workload": p.name, "m": p.m, "n": p.n, "Q": p.Q, "P": p.P, "iters": p.iters,
           "single_pass": plan.info()["single_pass"]}
    for key, graphs in (("plain_launches", False), ("graph_replay", True)):
        plan.set_graphs(graphs)
        plan.solve(g, p.iters)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v = plan.solve(g, p.iters)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        it = float(np.median(times))
        out[key] = {"iters_per_s": round(p.iters / it, 1), "us_per_iter": round(it / p.iters * 1e6, 2)}
    vn = v.cpu().numpy()
    out["nmse_vs_truth"] = float(np.linalg.norm(vn - p.u_true) ** 2 / np.linalg.norm(p.u_true) ** 2)
    print(f"[bench] 256x4096: plain {out['plain_launches']['iters_per_s']} it/s, graphs "
          f"{out['graph_replay']['iters_per_s']} it/s", file=sys.stderr, flush=True)
    plan.close()
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16
PARITY_ITERS = 4                 # iterations of the full-size parity points of the precision forms


def block_geometry(m: int, n: int, Q: int, P: int, direct: bool = False) -> dict:
    """Sizes the algorithmic byte counts need for equal splits (the first m % Q
    row blocks one row longer, likewise columns): the Gram matrices are
    m_i x m_i, or n_j x n_j in the direct form."""
    if direct:
        sizes, mult = [n // P + (1 if j < n % P else 0) for j in range(P)], Q
    else:
        sizes, mult = [m // Q + (1 if i < m % Q else 0) for i in range(Q)], P
    tiles = [(s_ + 63) // 64 for s_ in sizes]
    return {"m": m, "n": n,
            "ginv_packed": int(sum(T * (T + 1) // 2 * 4096 for T in tiles) * mult),
            "gram_parts": int(sum(T * T for T in tiles) * mult),
            "gram_parts_patch": int(sum(T * ((T + 3) // 4 + 1) for T in tiles) * mult)}


def model_times(A, m: int, n: int, Q: int, P: int, coef=None):
    """(setup s, iteration s) of the library's timing model (admm_choose_split)
    for split (Q, P), from admm_split_cost's features and the coefficients
    (built-in when None)."""
    c = A.split_cost(m, n, Q, P)
    k = A.model_coefficients() if coef is None else coef
    h = c["h_bytes"]
    hz = h * c["slab_load"] if c["single_pass"] else 0.0
    edge = c["max_block_cols"] if c["direct"] else c["max_block_rows"]
    fs = [c["setup_fp64_flops"], c["gram_span"], -(-int(edge) // 64), Q * P, 1.0]
    fi = [hz if c["slab_threads"] == 512 else 0.0, hz if c["slab_threads"] == 1024 else 0.0,
          c["bytes_per_iteration"] - h if c["single_pass"] else c["bytes_per_iteration"], Q * P, 1.0]
    return float(np.dot(fs, k[:5])), float(np.dot(fi, k[5:]))


def split_model(A, m: int, n: int, Q: int, P: int, coef=None) -> dict:
    """Modelled setup and iteration times of a split next to its exchange count."""
    c = A.split_cost(m, n, Q, P)
    su, it = model_times(A, m, n, Q, P, coef)
    return {"exchange_elements": int(c["exchange_elements"]), "model_setup_ms": round(su * 1e3, 2),
            "model_iter_us": round(it * 1e6, 1)}


CANDIDATES = (1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32)


def sweep_splits(torch, A, p, H, g, K: int) -> dict:
    """Every candidate equal split of the chooser: setup (plan construction
    with its workspace) and one K-iteration solve from zero after a 5-iteration
    warm-up, wall-clock around synchronisations."""
    out = {}
    for Q in CANDIDATES:
        for P in CANDIDATES:
            if Q > p.m or P > p.n:
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = A.Plan(H, Q, P, p.rho, p.lam)
            torch.cuda.synchronize()
            su = time.perf_counter() - t0
            plan.solve(g, 5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.solve(g, K)
            torch.cuda.synchronize()
            out[(Q, P)] = (su, time.perf_counter() - t0)
            plan.close()
            del plan
    torch.cuda.empty_cache()
    return out


def bench_chooser(torch, A, p, H, g, K: int) -> dict:
    """The split chooser against measurement (Sec. IV; next to the paper's
    splittings): every candidate is set up and run for K iterations, and the
    picks of the model with its built-in coefficients, with coefficients
    calibrated on this device (admm_calibrate), and of the measuring chooser
    (model shortlist of 6 timed on the device) are compared with the best
    measured total."""
    t0 = time.perf_counter()
    coef = A.calibrate(H, g)
    cal_s = time.perf_counter() - t0
    picks = {"model_builtin": A.choose_split(p.m, p.n, K)[:2],
             "model_calibrated": A.choose_split(p.m, p.n, K, coef=coef)[:2]}
    t0 = time.perf_counter()
    picks["measured_shortlist_6"] = A.choose_split_measure(H, g, K, coef=coef, shortlist_len=6)[:2]
    meas_s = time.perf_counter() - t0
    sw = sweep_splits(torch, A, p, H, g, K)
    tot = {k: v[0] + v[1] for k, v in sw.items()}
    best = min(tot, key=tot.get)
    res = {"iters": K, "candidates": len(sw), "best_measured": {"split": f"{best[0]}x{best[1]}",
                                                                "total_ms": round(tot[best] * 1e3, 2)},
           "calibration_s": round(cal_s, 3), "measuring_chooser_s": round(meas_s, 3),
           "calibrated_coefficients": [float(x) for x in coef], "picks": {}}
    for name, (Q, P) in picks.items():
        su, it = model_times(A, p.m, p.n, Q, P, coef if name != "model_builtin" else None)
        res["picks"][name] = {"split": f"{Q}x{P}", "measured_total_ms": round(tot[(Q, P)] * 1e3, 2),
                              "over_best": round(tot[(Q, P)] / tot[best], 3),
                              "model_total_ms": round((su + K * it) * 1e3, 2)}
    # the model's error over all candidates (calibrated coefficients)
    errs = []
    for (Q, P), t in tot.items():
        su, it = model_times(A, p.m, p.n, Q, P, coef)
        errs.append(abs(su + K * it - t) / t)
    res["model_rel_error_calibrated"] = {"mean": round(float(np.mean(errs)), 3), "max": round(float(np.max(errs)), 3)}
    res["sweep_ms"] = {f"{Q}x{P}": [round(v[0] * 1e3, 2), round(v[1] * 1e3, 2)] for (Q, P), v in sorted(sw.items())}
    return res


def bench_full_splits(args, torch, A, prob, H, g, steps: int = 300, warmup: int = 300):
    """The other two methods on the full matrix: consensus only (Q = 4, P = 1,
    1536 x 32000 blocks) and sectioning only (Q = 1, P = 8, 6144 x 4000
    blocks, taller than wide; Q = 1, P = 32, 6144 x 1000 blocks, which take
    the direct x-update), complex64, same rho and lambda."""
    rows = []
    for Q, P in ((4, 1), (1, 8), (1, 32)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = A.Plan(H, Q, P, prob.rho, prob.lam)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        plan.solve(g, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v, hist = plan.solve(g, steps, history=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        info = plan.info()
        algo = algorithmic_bytes(block_geometry(prob.m, prob.n, Q, P, info["direct"]), P, Q, info["chunks"], "c64",
                                 "c64", info["gram_patches"] > 0, info["slab_workgroups"])
        vn = v.cpu().numpy()
        hs = hist.cpu().numpy()
        mi, nj = -(-prob.m // Q), -(-prob.n // P)
        rows.append({
            "split": f"{Q}x{P}", "block": f"{mi}x{nj}", "value": round(steps / el, 1), "unit": "iters/s",
            "setup_ms": round(setup * 1e3, 1), "iteration_gbs": round(iteration_bytes(algo, info) * steps / el / 1e9, 1),
            "algo_bytes_per_iteration": iteration_bytes(algo, info), "single_pass": info["single_pass"],
            "direct": info["direct"], "inverse_gb": round(info["ginv_bytes"] / 1e9, 3),
            "nmse_vs_truth": float(np.linalg.norm(vn - prob.u_true) ** 2 / np.linalg.norm(prob.u_true) ** 2),
            "residuals_last": [float(x) for x in hs[-1]],
            "iter_us": round(el / steps * 1e6, 1), **split_model(A, prob.m, prob.n, Q, P),
        })
        plan.close()
        print(f"[bench] full matrix {Q}x{P}: setup {setup * 1e3:.1f} ms, {steps / el:.1f} iterations/s",
              file=sys.stderr, flush=True)
    return {"workload": prob.name.split("_")[0], "iters": steps, "warmup": warmup, "splits": rows}


# The paper's timing table (Sec. VI): per splitting, inversion time (ms), 50
# iterations (ms) and total imaging time (s), one Titan V under MATLAB R2017b
# at 2160 x 22500 (precision not stated).  Quoted as context only.
PAPER_TABLE_TIMES = {(4, 1): (196.0, 616.0, 0.812), (1, 3): (381.0, 639.0, 1.020), (4, 3): (248.0, 1171.0, 1.419)}


def bench_paper_table(args, torch, A, W, dev, reps: int = 5):
    """The paper's timing-table workload on one MI355X: 2160 x 22500, the three
    splittings, setup (FP64 Gram, Cholesky and inverse, the paper's inversion
    step) and 50 iterations timed apart, complex64; then the splits the cost
    model chooses for 50 iterations, without and with a limit of 10000
    exchanged elements per node."""
    p = W.paper_table_imaging(seed=args.seed)
    H = torch.from_numpy(p.H).to(dev)
    g = torch.from_numpy(p.g).to(dev)
    K = W.PAPER_TABLE_ITERS
    rows = []
    chosen = [A.choose_split(p.m, p.n, K, max_exchange=lim)[:2] for lim in (0.0, 10000.0)]
    splits = list(W.PAPER_TABLE_SPLITS) + [(1, 32)]   # and the direct x-update's 2160 x 703 blocks
    for s in chosen:
        if s not in splits:
            splits.append(s)
    for Q, P in splits:
        A.Plan(H, Q, P, p.rho, p.lam).close()   # first build of this split, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = A.Plan(H, Q, P, p.rho, p.lam)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        plan.solve(g, K)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v, hist = plan.solve(g, K, history=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        it = float(np.median(times))
        info = plan.info()
        algo = algorithmic_bytes(block_geometry(p.m, p.n, Q, P, info["direct"]), P, Q, info["chunks"], "c64", "c64",
                                 info["gram_patches"] > 0, info["slab_workgroups"])
        vn = v.cpu().numpy()
        hs = hist.cpu().numpy()
        mi, nj = -(-p.m // Q), -(-p.n // P)
        rows.append({
            "split": f"{Q}x{P}", "block": f"{mi}x{nj}",
            "inverse": f"{nj}x{nj}" if info["direct"] else f"{mi}x{mi}", "direct": info["direct"],
            "setup_ms": round(setup * 1e3, 2), "iters_ms": round(it * 1e3, 3),
            "total_ms": round((setup + it) * 1e3, 2), "iters_per_s": round(K / it, 1),
            "iteration_gbs": round(iteration_bytes(algo, info) * K / it / 1e9, 1),
            "single_pass": info["single_pass"],
            "nmse_vs_truth": float(np.linalg.norm(vn - p.u_true) ** 2 / np.linalg.norm(p.u_true) ** 2),
            "residuals_first_last": [[float(x) for x in hs[0]], [float(x) for x in hs[-1]]],
            **split_model(A, p.m, p.n, Q, P),
        })
        if (Q, P) in PAPER_TABLE_TIMES:
            ps, pi, pt = PAPER_TABLE_TIMES[(Q, P)]
            rows[-1]["paper_titan_v"] = {"inversion_ms": ps, "iters_ms": pi, "total_s": pt}
        if (Q, P) in chosen:
            rows[-1]["chosen_by_model"] = {"max_exchange": 0 if (Q, P) == chosen[0] else 10000}
        plan.close()
        print(f"[bench] paper table {Q}x{P}: setup {setup * 1e3:.1f} ms, {K} iterations {it * 1e3:.2f} ms",
              file=sys.stderr, flush=True)
    chooser = bench_chooser(torch, A, p, H, g, K)
    print(f"[bench] chooser on {p.m}x{p.n}, {K} iterations: best measured {chooser['best_measured']}, picks "
          + ", ".join(f"{k} {v['split']} x{v['over_best']}" for k, v in chooser["picks"].items()),
          file=sys.stderr, flush=True)
    del H, g
    torch.cuda.empty_cache()
    return {"workload": "cra2160x22500", "m": p.m, "n": p.n, "rho": p.rho, "lam_ratio": 0.02, "iters": K,
            "dtype": "c64", "timing": f"setup of a second build; iterations: median of {reps} solves from zero",
            "paper_hardware": "one Titan V, MATLAB R2017b (context, not a target)", "splits": rows,
            "chooser": chooser}


def bench_batch(args, torch, A, W, dev):
    """Batched multi-scene form: S scenes (seeds 1000..) sharing the 6144 x
    32000 instrument, frequency subsets of 12..24 tiles, Q in {2,4,8}, P=8,
    300 iterations each, solved together with hipGraph replay; compared with
    the plain complex64 solver run one scene at a time on a subset."""
    t = time.perf_counter()
    b = W.batch_scenes(S=args.batch_scenes)
    gen_s = time.perf_counter() - t
    H0 = torch.from_numpy(b.H0).to(dev)
    g = torch.from_numpy(np.concatenate(b.g)).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    bb = A.Batch(H0, b.tile_rows, b.tiles, b.cuts, b.phases, b.P, b.rho, b.lam)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    info = bb.info()
    print(f"[bench] batch: {b.S} scenes generated in {gen_s:.1f}s, setup {setup_s:.2f}s, "
          f"{info['scene_tiles']} scene-tiles", file=sys.stderr, flush=True)
    K = args.batch_iters or b.iters
    bb.solve(g, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = bb.solve(g, K, graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # per-kernel event timing on a short run without the graph
    bb.profile(True)
    bb.solve(g, 10, graph=False)
    prof = {bb.KERNELS[k]: bb.profile_read(k) for k in bb.KERNELS}
    bb.profile(False)
    n, NST = b.H0.shape[1], info["scene_tiles"]
    cmacs = NST * b.tile_rows * n                      # complex MACs of one GEMM pass
    mfma_flop = 2 * 12 * cmacs                         # 3-term split: 12 real MFMA MACs per complex MAC
    algo_flop = 8 * cmacs                              # the product itself: 8 real flops per complex MAC
    kern = {}
    for name, (ms, cnt) in prof.items():
        kern[name] = {"avg_us": round(ms / max(cnt, 1) * 1e3, 2), "launches": cnt}
    for name in ("k_bgemm_n", "k_bgemm_h"):
        sec = kern[name]["avg_us"] * 1e-6
        kern[name]["mfma_tflops"] = round(mfma_flop / sec / 1e12, 1)
        kern[name]["mfma_frac"] = round(mfma_flop / sec / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)
        kern[name]["algo_tflops"] = round(algo_flop / sec / 1e12, 1)
        kern[name]["algo_frac"] = round(algo_flop / sec / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)
        kern[name]["mfma_flop_per_pass"] = mfma_flop
        kern[name]["h0_gbs"] = round(b.H0.size * 4 / sec / 1e9, 1)
    gsec = kern["k_gram"]["avg_us"] * 1e-6
    kern["k_gram"]["gbs"] = round(info["ginv_bytes"] / gsec / 1e9, 1)
    vn = v.cpu().numpy()
    nmse_b = [float(np.linalg.norm(vn[s] - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2) for s in range(b.S)]
    # plain complex64 solver, one scene at a time, on the first scenes
    seq = []
    for s in range(min(args.batch_seq, b.S)):
        rows = torch.from_numpy(b.rows(s)).to(dev)
        ph = torch.from_numpy(b.phases[s]).to(dev)
        Hs = (H0.index_select(0, rows) * ph[:, None]).contiguous()
        gs = torch.from_numpy(b.g[s]).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = A.Plan(Hs, len(b.cuts[s]) - 1, b.P, b.rho, b.lam[s], b.row_off(s))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vs = plan.solve(gs, K)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        seq.append((t2 - t0, float(np.linalg.norm(vs.cpu().numpy() - b.u_true[s]) ** 2 /
                                   np.linalg.norm(b.u_true[s]) ** 2), t2 - t1))
        plan.close()
        del Hs, plan
    seq_t = float(np.mean([x[0] for x in seq])) if seq else float("nan")
    seq_it = float(np.mean([x[2] for x in seq])) if seq else float("nan")
    res = {
        "workload": b.name, "scenes": b.S, "iters": K, "value": round(b.S / el, 2),
        "unit": "scenes/s (300 iterations each, setup apart)",
        "value_with_setup": round(b.S / (el + setup_s), 2),
        "ms_per_batched_iteration": round(el / K * 1e3, 3), "setup_s": round(setup_s, 2),
        "scene_tiles": NST, "gemm_choice": {"fwd_rows_per_wg": info["fwd_rows_per_wg"], "fwd_kchunks": info["fwd_kchunks"],
                                  "adj_cols_per_wg": info["adj_cols_per_wg"]}, "autotune": bb.tuning(),
        "kernels": kern, "ginv_gb": round(info["ginv_bytes"] / 1e9, 2),
        "nmse_mean": float(np.mean(nmse_b)),
        "plain_one_at_a_time": {
            "scenes": len(seq), "value": round(1.0 / seq_it, 2) if seq else None,
            "unit": "scenes/s (300 iterations each, setup apart)",
            "value_with_setup": round(1.0 / seq_t, 2) if seq else None,
            "nmse_mean": float(np.mean([x[1] for x in seq])) if seq else None,
            "batched_nmse_mean_same_scenes": float(np.mean(nmse_b[:len(seq)])) if seq else None,
        },
    }
    bb.close()
    del bb
    torch.cuda.empty_cache()
    # the same batch with the bfloat16 copy of the scene inverses
    t = time.perf_counter()
    bb = A.Batch(H0, b.tile_rows, b.tiles, b.cuts, b.phases, b.P, b.rho, b.lam, inverse="bf16")
    torch.cuda.synchronize()
    setup16 = time.perf_counter() - t
    bb.solve(g, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v16 = bb.solve(g, K, graph=True)
    torch.cuda.synchronize()
    el16 = time.perf_counter() - t0
    bb.profile(True)
    bb.solve(g, 10, graph=False)
    k16 = {bb.KERNELS[k]: round(bb.profile_read(k)[0] / max(bb.profile_read(k)[1], 1) * 1e3, 2) for k in bb.KERNELS}
    bb.profile(False)
    v16n = v16.cpu().numpy()
    nmse16 = [float(np.linalg.norm(v16n[s] - b.u_true[s]) ** 2 / np.linalg.norm(b.u_true[s]) ** 2) for s in range(b.S)]
    res["inverse_bf16"] = {
        "value": round(b.S / el16, 2), "unit": "scenes/s (300 iterations each, setup apart)",
        "value_with_setup": round(b.S / (el16 + setup16), 2), "ms_per_batched_iteration": round(el16 / K * 1e3, 3),
        "setup_s": round(setup16, 2), "kernels_avg_us": k16,
        "gram_gbs": round(info["ginv_bytes"] / 2 / (k16["k_gram"] * 1e-6) / 1e9, 1),
        "nmse_mean": float(np.mean(nmse16)),
        "rel_diff_vs_fp32_inverse": float(np.linalg.norm(v16n - vn) / np.linalg.norm(vn)),
    }
    print(f"[bench] batch, bf16 inverse: {res['inverse_bf16']['value']} scenes/s", file=sys.stderr, flush=True)
    bb.close()
    del H0, g, bb
    torch.cuda.empty_cache()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the bf16 / fp8 storage forms")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched multi-scene form")
    ap.add_argument("--no-paper-table", action="store_true", help="skip the paper's timing-table workload")
    ap.add_argument("--no-splits", action="store_true", help="skip the consensus-only and sectioning-only splits")
    ap.add_argument("--paper-table-only", action="store_true", help="measure only the paper's timing-table workload")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--batch-seq", type=int, default=8, help="scenes solved one at a time for comparison")
    ap.add_argument("--batch-iters", type=int, default=0,
                    help="iterations of the batched solves (0: the workload's 300; counter runs use a few)")
    ap.add_argument("--summarise-mfma", nargs=2, metavar=("COUNTER_CSV", "TRACE_CSV"),
                    help="write profiles/mfma_<batch workload>.md from an MFMA counter run and its kernel trace")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-small", action="store_true", help="skip the 256 x 4096 workload")
    ap.add_argument("--small-only", action="store_true", help="measure only the 256 x 4096 workload")
    ap.add_argument("--no-convergence", action="store_true",
                    help="skip the KKT violation and NMSE at growing iteration counts")
    ap.add_argument("--no-form-oracle", action="store_true",
                    help="skip the oracle runs on the dequantised bf16 / fp8 matrices")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--batch-only", action="store_true", help="measure only the batched multi-scene form")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the region without kernel events (kernel timings from a second run)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of MIB MiB (counter calibration)")
    ap.add_argument("--summarise-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_*.json from two rocprofv3 --pmc runs and exit (no GPU)")
    ap.add_argument("--probe-mib", type=int, default=1024)
    ap.add_argument("--command", default="", help="counter command recorded in the traffic summary")
    args = ap.parse_args(argv)

    if args.summarise_mfma:
        print(summarise_mfma(args.summarise_mfma[0], args.summarise_mfma[1], args.command))
        return 0
    if args.summarise_traffic:
        import workloads as W
        for p in summarise_traffic(args.summarise_traffic[0], args.summarise_traffic[1], args.probe_mib,
                                   W.full_imaging_name(), args.command):
            print(p)
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver keeps every block of the split on a single "
              "MI355X and has no multi-GPU path (--gpus must be 1).", file=sys.stderr)
        return 2

    import torch

    import paper_1811_05571_amd as A
    import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe:
        copy_probe(torch, dev, args.copy_probe)
    if args.batch_only:
        print(json.dumps({"batch": bench_batch(args, torch, A, W, dev)}), flush=True)
        return 0
    if args.paper_table_only:
        print(json.dumps({"paper_table": bench_paper_table(args, torch, A, W, dev)}), flush=True)
        return 0
    if args.small_only:
        print(json.dumps({"small_256x4096": bench_small(args, torch, A, W, dev)}), flush=True)
        return 0
    t = time.perf_counter()
    prob = W.full_imaging(seed=args.seed)
    gen_s = time.perf_counter() - t
    print(f"[bench] generated {prob.name} m={prob.m} n={prob.n} Q={prob.Q} P={prob.P} rho={prob.rho} "
          f"lam={prob.lam:.4g} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    H = torch.from_numpy(prob.H).to(dev)
    g = torch.from_numpy(prob.g).to(dev)
    torch.cuda.synchronize()

    geo = block_geometry(prob.m, prob.n, prob.Q, prob.P)
    workload = prob.name

    def measure(storage: str, steps: int, warmup: int, inverse: str = "c64", before=None):
        t = time.perf_counter()
        plan = A.Plan(H, prob.Q, prob.P, prob.rho, prob.lam, storage=storage, inverse=inverse)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        info = plan.info()
        # another measurement on the same plan first (untimed here; its solves
        # start from zero like the timed one)
        before_res = before(plan) if before is not None else None
        if warmup > 0:   # with the residual history, as timed (its first use costs a one-off allocation)
            plan.solve(g, warmup, history=True)
        # kernel events (on the dispatch packets) on every 10th iteration of the timed region
        plan.profile(0 if args.no_kernel_events else PROFILE_EVERY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v, hist = plan.solve(g, steps, history=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if args.no_kernel_events:   # kernel timings from a separate run of the same length
            plan.profile(PROFILE_EVERY)
            plan.solve(g, steps)
        prof = {A.KERNEL_NAMES[k]: plan.profile_read(k) for k in A.KERNEL_NAMES}
        plan.profile(False)
        algo = algorithmic_bytes(geo, prob.P, prob.Q, info["chunks"], storage, inverse, info["gram_patches"] > 0,
                                 info["slab_workgroups"])
        kern = {}
        for name, (ms, cnt) in prof.items():
            if cnt == 0:
                continue
            avg_ms = ms / max(cnt, 1)
            kern[name] = {"avg_us": round(avg_ms * 1e3, 3), "launches": cnt, "algo_bytes": algo[name],
                          "gbs": round(algo[name] / (avg_ms * 1e-3) / 1e9, 1)}
        dominant = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
        dk = kern[dominant]
        v_np = v.cpu().numpy()
        res = {
            "plan": plan, "v": v, "elapsed": elapsed, "setup_s": setup_s, "info": info, "kern": kern,
            "before": before_res,
            "dominant": dominant,
            "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(dk["gbs"] / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic(dominant, f"{workload}_{storage}") if inverse == "c64" else None,
                         "algo_bytes_per_launch": dk["algo_bytes"], "avg_launch_us": dk["avg_us"]},
            "iteration_gbs": round(iteration_bytes(algo, info) * steps / elapsed / 1e9, 1),
            "nmse": float(np.linalg.norm(v_np - prob.u_true) ** 2 / np.linalg.norm(prob.u_true) ** 2),
            "kkt": plan.kkt(g, v), "final_residuals": [float(x) for x in hist[-1].cpu().numpy()],
        }
        print(f"[bench] {storage} (inverse {inverse}): setup {setup_s * 1e3:.1f} ms, {steps} iterations in "
              f"{elapsed * 1e3:.1f} ms", file=sys.stderr, flush=True)
        return res

    # The convergence leg's solves (about 3 s of the same iteration, back to
    # back) run on the headline plan before its warm-up and timed region,
    # which then start with the GPU at the clocks it holds under this load,
    # as in a long solve; their KKT and NMSE are evaluated afterwards.
    main = measure("c64", args.steps, args.warmup,
                   before=None if args.no_convergence else
                   (lambda pl: convergence_run(pl, g, CONVERGENCE_CHECKPOINTS)))
    plan = main["plan"]
    # the same solve replaying captured graphs of 10 iterations (no kernel events)
    plan.set_graphs(True)
    plan.solve(g, max(args.steps, 10), history=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve(g, args.steps, history=True)
    torch.cuda.synchronize()
    graph_el = time.perf_counter() - t0
    out = {
        "metric": "ADMM iters/s", "value": round(args.steps / main["elapsed"], 2), "unit": "iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main["elapsed"] / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": workload, "m": prob.m, "n": prob.n, "Q": prob.Q, "P": prob.P,
                   "rho": prob.rho, "lam_ratio": 0.02, "storage": "c64", "parallelism": "single-gpu"},
        "roofline": main["roofline"],
        "iteration_gbs": main["iteration_gbs"],
        "graph_replay": {"value": round(args.steps / graph_el, 2), "ms_per_step": round(graph_el / args.steps * 1e3, 4),
                         "note": "same solve replaying captured graphs of 10 iterations, no kernel events"},
        "single_pass": main["info"]["single_pass"],
        "kernels": main["kern"],
        "setup_ms": round(main["setup_s"] * 1e3, 1),
        "nmse_vs_truth": main["nmse"], "kkt_violation": main["kkt"],
        "final_residuals": main["final_residuals"],
    }
    if main["before"] is not None:
        out["convergence"] = convergence_eval(plan, g, prob, main["before"])
    form_plans = {}
    if not args.no_forms:
        forms = {}
        v_ref = main["v"].cpu().numpy()
        for key, storage, inverse in (("bf16", "bf16", "c64"), ("fp8", "fp8", "c64"),
                                      ("c64_inverse_bf16", "c64", "bf16"), ("fp8_inverse_bf16", "fp8", "bf16")):
            r = measure(storage, args.steps, args.warmup, inverse)
            vq = r["v"].cpu().numpy()
            # reconstruction quality after the workload's 300 iterations
            v300 = r["plan"].solve(g, prob.iters)
            v300n = v300.cpu().numpy()
            forms[key] = {
                "storage": storage, "inverse": inverse,
                "value": round(args.steps / r["elapsed"], 2), "unit": "iters/s",
                "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 4), "roofline": r["roofline"],
                "iteration_gbs": r["iteration_gbs"], "kernels": r["kern"], "setup_ms": round(r["setup_s"] * 1e3, 1),
                "after_300_iterations": {
                    "nmse_vs_truth": float(np.linalg.norm(v300n - prob.u_true) ** 2
                                           / np.linalg.norm(prob.u_true) ** 2),
                    "kkt_violation": r["plan"].kkt(g, v300)},
                "rel_diff_vs_c64_image": float(np.linalg.norm(vq - v_ref) / max(np.linalg.norm(v_ref), 1e-300)),
            }
            if storage != "c64" and inverse == "c64":
                form_plans[storage] = r["plan"]
                continue
            r["plan"].close()
            del r
        out["forms"] = forms
    if not args.no_adjoint:
        # reverse mode of K = 100 unrolled iterations, checkpoint every 10
        K, C = 100, 10
        plan.set_lambda(prob.lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vK = plan.solve(g, K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vR, tape = plan.solve_record(g, K, C)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ut = torch.from_numpy(prob.u_true.astype(np.complex64)).to(dev)
        gv = 2 * (vR - ut)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gg, dl, dr = plan.backward(g, gv, tape)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        out["adjoint"] = {
            "iters": K, "checkpoint_interval": C, "forward_ms": round((t1 - t0) * 1e3, 2),
            "record_ms": round((t2 - t1) * 1e3, 2), "backward_ms": round((t4 - t3) * 1e3, 2),
            "backward_over_forward": round((t4 - t3) / (t1 - t0), 3), "tape_mb": round(tape.numel() / 1e6, 1),
            "dL_dlambda": dl, "dL_drho": dr, "grad_g_norm": float(torch.linalg.vector_norm(gg).item()),
        }
        print(f"[bench] adjoint: forward {out['adjoint']['forward_ms']} ms, backward "
              f"{out['adjoint']['backward_ms']} ms", file=sys.stderr, flush=True)
    if not args.no_small:
        out["small_256x4096"] = bench_small(args, torch, A, W, dev)
    if not args.no_splits:
        out["full_splits"] = bench_full_splits(args, torch, A, prob, H, g)
    del H
    if not args.no_batch:
        out["batch"] = bench_batch(args, torch, A, W, dev)
    if not args.no_paper_table:
        out["paper_table"] = bench_paper_table(args, torch, A, W, dev)

    out["attainable"] = attainable_bandwidth(torch, dev)
    if not args.no_cpu:
        print(f"[bench] oracle CPU baseline: setup + {args.cpu_iters} iterations", file=sys.stderr, flush=True)
        kp = min(PARITY_ITERS, args.cpu_iters)
        cb = cpu_baseline(prob, args.cpu_iters, keep=(kp,))
        # parity at full size on the same sample: GPU from zero, same iteration counts
        vg = plan.solve(g, args.cpu_iters).cpu().numpy()
        err = float(np.linalg.norm(vg - cb["v"]) / max(np.linalg.norm(cb["v"]), 1e-300))
        out["cpu_baseline"] = {
            "value": round(1.0 / cb["iter_s"], 4), "unit": "iters/s", "cores": cb["threads"], "kind": "oracle",
            "form": "push-through (two products with each block per iteration)",
            "sample": f"{prob.name}: oracle setup ({cb['setup_s']:.1f} s, not in value) then "
                      f"{cb['iters']} iterations from zero, FP64 complex128, push-through form, {cb['blas']} "
                      f"BLAS with {cb['threads']} threads on {cb['affinity']} available cores",
            "setup_s": round(cb["setup_s"], 2),
        }
        out["parity_at_full_size"] = {"iters": args.cpu_iters, "rel_err_vs_oracle": err}
        # precision forms against the oracle after kp iterations: on the
        # dequantised H (arithmetic error) and on the complex64 H (total)
        if form_plans and not args.no_form_oracle:
            from oracle import quant as QZ
            v64 = cb["kept"][kp]
            fe = {}
            for storage, fplan in form_plans.items():
                vq = fplan.solve(g, kp).cpu().numpy()
                print(f"[bench] oracle on the dequantised {storage} H: {kp} iterations", file=sys.stderr,
                      flush=True)
                cq = cpu_baseline(prob, kp, keep=(kp,), H=QZ.dequantise(prob.H, storage))
                rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
                fe[storage] = {"iters": kp, "rel_err_vs_oracle_dequantised_H": rel(vq, cq["kept"][kp]),
                               "rel_err_vs_oracle_c64_H": rel(vq, v64)}
                fplan.close()
            out["forms_vs_oracle"] = fe
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
