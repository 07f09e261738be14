#!/usr/bin/env python3
"""Throughput of the streamed GWAS GLS hot path on one MI355X.

One step = one whole study: setup (M, Cholesky, inverse factor, covariate
terms), every SNP block through the triangular product, the per-SNP products
and p x p solves, and the results copied to host memory.  The SNP matrix is
resident in HBM when the timed region starts (the PCIe-inclusive streamed
rate is reported separately with --stream).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c1_n10k_m100k]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SNPs/sec (GLS solves/s) at n=10k,p=4; TRSM TFLOP/s vs MFMA peak"
PEAK_TFLOPS = {"fp64": 78.6, "fp32_ir": 157.3, "fp16_ir": 2500.0, "bf16_ir": 2500.0}


# HBM traffic of the dominant kernel per full 8,192-SNP launch at n = 10,000, from
# two rocprofv3 --pmc runs (FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000, factors
# from a 1 GiB device copy; summary in profiles/).  Valid only while the
# kernel source is the one those counters were taken on.
TRAFFIC_RECORD = {"kernel_sha1": "32a87d13753b7a1e", "n": 10000, "block_cols": 8192, "bytes_per_launch": 29.54e9}


def kernel_hash() -> str:
    """Hash of the sources of the per-block product kernel (traffic records apply to one version)."""
    import hashlib
    h = hashlib.sha1()
    for f in ("gemm_f64.hpp", "gemm_f64_dma.hpp", "lds_dma.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1302_4332_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    """CPU model and the BLAS library numpy uses, for the CPU baseline."""
    d = {"cpu_count": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    d["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import threadpoolctl
        blas = [x for x in threadpoolctl.threadpool_info() if x.get("user_api") == "blas"]
        if blas:
            d["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')} ({blas[0].get('num_threads')} threads)"
    except Exception:
        pass
    return d


def blas_threads() -> int:
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n = [d.get("num_threads", 0) for d in info if d.get("user_api") == "blas"]
        return int(max(n)) if n else (os.cpu_count() or 1)
    except Exception:
        return os.cpu_count() or 1


def measure_forms(args, st, Phi_d, XL_d, y_d, X_d, m, dev):
    """Mixed-precision forms on the same workload, and the adjoint on the
    n = 4,096 differentiation study; one timed study each."""
    import torch

    from oracle import gls_oracle as O
    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext, GLSFunction, t2_loss

    w = st.w
    n, p, bc, h2 = w.n, w.p, w.block_cols, w.h2
    res = {}
    # oracle on a sample of SNPs (first 512 and the ragged tail) for the error of each form
    ost = O.Study(st.Phi, h2, st.XL, st.y)
    samp = np.r_[np.arange(512), np.arange(m - 64, m)]
    ref = ost.block(np.concatenate([st.snps(0, 512), st.snps(m - 64, m)]).T)
    # error of b against the oracle after 0..4 refinement sweeps, on the sample
    Xs_d = torch.tensor(np.concatenate([st.snps(0, 512), st.snps(m - 64, m)]), device=dev)
    ok = ref["status"] == 0
    by_sweeps = {}
    for prec in ("fp32_ir", "fp16_ir", "bf16_ir"):
        errs = []
        for k in range(5):
            ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=Xs_d.shape[0], precision=prec, refine_sweeps=k)
            gb = ctx.block(Xs_d)[0].cpu().numpy()
            ctx.close()
            errs.append(float((np.max(np.abs(gb[ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)).max()))
        by_sweeps[prec] = errs
        log(f"{prec} max rel err of b after 0..4 sweeps: " + ", ".join(f"{e:.1e}" for e in errs))
    res["max_rel_err_b_by_sweeps"] = {"sweeps": [0, 1, 2, 3, 4], **by_sweeps,
                                      "sample": "SNPs [0, 512) and the last 64, against the oracle"}
    del Xs_d
    # the fewest sweeps that meet the 1e-8 bar on b (FP32 1, FP16 2, BF16 3),
    # and for FP16 and BF16 also the sweep counts that reach the FP64 level
    for prec, sweeps in (("fp32_ir", 1), ("fp16_ir", 2), ("fp16_ir", 3), ("bf16_ir", 3), ("bf16_ir", 4)):
        b_d = torch.empty((m, p), dtype=torch.float64, device=dev)
        s2_d = torch.empty(m, dtype=torch.float64, device=dev)
        v_d = torch.empty(m, dtype=torch.float64, device=dev)
        st_d = torch.empty(m, dtype=torch.int32, device=dev)

        def study(profile):
            ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=prec, refine_sweeps=sweeps)
            if profile:
                ctx.profile(True)
            for j0 in range(0, m, bc):
                j1 = min(m, j0 + bc)
                ctx.block_into(X_d[j0:j1], b_d[j0:j1], s2_d[j0:j1], v_d[j0:j1], st_d[j0:j1])
            ph = ctx.profile_read() if profile else None
            ctx.close()
            return ph

        study(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ph = study(True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        g = b_d.cpu().numpy()[samp]
        ok = ref["status"] == 0
        err = np.max(np.abs(g[ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)
        lp_ms, res_ms = ph["whiten"][1], ph["residual"][1]
        lp_flops = float(n) * n * m * (1 + sweeps)
        r_flops = float(n) * n * m * sweeps
        res[f"{prec}_{sweeps}sweeps"] = {
            "snps_per_s": m / (ms / 1e3), "ms_per_study": ms, "max_rel_err_b_sampled": float(err.max()),
            "lowp_tflops": lp_flops / (lp_ms / 1e3) / 1e12, "lowp_peak": PEAK_TFLOPS[prec],
            "fp64_residual_tflops": (r_flops / (res_ms / 1e3) / 1e12) if res_ms else None,
            "phases_ms": {k: v[1] for k, v in ph.items()}}
        log(f"{prec} x{sweeps}: {m / (ms / 1e3):,.0f} SNPs/s, max rel err {err.max():.2e}")
        del b_d, s2_d, v_d, st_d
    # adjoint on the differentiation study
    w3 = synth.WORKLOADS["c3_grad_n4096"]
    s3 = synth.make_study(w3)
    X3 = torch.tensor(s3.snps(0, w3.m), device=dev)
    Phi3, XL3, y3 = (torch.tensor(a, device=dev) for a in (s3.Phi, s3.XL, s3.y))
    for prec, sweeps in (("fp64", 0), ("fp32_ir", 2)):
        def fwd_bwd():
            yt = y3.clone().requires_grad_(True)
            Xt = X3.clone().requires_grad_(True)
            h2t = torch.tensor(w3.h2, dtype=torch.float64, device=dev, requires_grad=True)
            b, s2, v = GLSFunction.apply(yt, Xt, h2t, Phi3, XL3, w3.block_cols, prec, sweeps)
            t2_loss(b, s2, v).backward()
            return h2t.grad
        fwd_bwd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gh = fwd_bwd()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res[f"adjoint_c3_{prec}"] = {"workload": w3.name, "ms_fwd_bwd": ms, "snps_per_s": w3.m / (ms / 1e3),
                                     "h2_grad": float(gh)}
        log(f"adjoint {prec}: {ms:.1f} ms forward+backward")
    return res


def measure_bytes(args, st, Phi_d, XL_d, y_d, X_d, m, dev, b_fp64_host):
    """Genotype bytes: the int8-slice product (FP64-accurate) with the SNP
    matrix resident in HBM, and the streamed rates from pinned host memory
    and from a file, as bytes (1 byte per sample instead of 8) and as packed
    2-bit dosages (a quarter byte per sample)."""
    import tempfile

    import torch

    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext

    w = st.w
    n, p, bc, h2 = w.n, w.p, w.block_cols, w.h2
    res = {}
    G_d = X_d.to(torch.uint8)
    b_d = torch.empty((m, p), dtype=torch.float64, device=dev)
    s2_d = torch.empty(m, dtype=torch.float64, device=dev)
    v_d = torch.empty(m, dtype=torch.float64, device=dev)
    st_d = torch.empty(m, dtype=torch.int32, device=dev)

    ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision="int8_emu")

    def study(profile):
        if profile:
            ctx.profile(True)
        for j0 in range(0, m, bc):
            j1 = min(m, j0 + bc)
            ctx.block_u8_into(G_d[j0:j1], b_d[j0:j1], s2_d[j0:j1], v_d[j0:j1], st_d[j0:j1])
        return ctx.profile_read() if profile else None

    study(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ph = study(True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    g = b_d.cpu().numpy()
    ref = b_fp64_host.numpy()
    ok = np.isfinite(ref).all(axis=1)
    rel = np.max(np.abs(g[ok] - ref[ok]), axis=1) / np.max(np.abs(ref[ok]), axis=1)
    wl, wms = ph["whiten"]
    res["int8_emu_hbm"] = {
        "snps_per_s": m / (ms / 1e3), "ms_per_study": ms, "slices": 8,
        "product_ms": wms, "product_fp64_equiv_tflops": float(n) * n * m / (wms / 1e3) / 1e12,
        "int8_tops": 8.0 * n * n * m / (wms / 1e3) / 1e12, "int8_peak_tops": 5000.0,
        "max_rel_diff_vs_fp64_path": float(rel.max()),
        "note": "same study, SNPs as bytes; product from exact int8 slice products (FP64-level accuracy)"}
    log(f"int8 emulation: {m / (ms / 1e3):,.0f} SNPs/s, product {wms:.1f} ms, max rel diff vs FP64 path {rel.max():.2e}")
    del b_d, s2_d, v_d, st_d
    G_h = torch.empty((m, n), dtype=torch.uint8).pin_memory()
    G_h.copy_(G_d)
    del G_d
    G2_h = torch.from_numpy(synth.pack_dosages_2bit(G_h.numpy())).pin_memory()
    inputs = {"u8": (G_h, False), "u2": (G2_h, True)}
    for fmt, (H, packed) in inputs.items():
        for prec in ("fp64", "int8_emu"):
            ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=prec)
            ctx.stream(H, packed=packed)
            (_, _, _, _), ss = ctx.stream(H, packed=packed)
            res[f"stream_{fmt}_{prec}"] = {"snps_per_s": m / (ss.wall_ms / 1e3), "wall_ms": ss.wall_ms,
                                           "compute_ms": ss.compute_ms,
                                           "h2d_GBps": ss.h2d_bytes / (ss.wall_ms / 1e3) / 1e9}
            log(f"stream {fmt} {prec}: {m / (ss.wall_ms / 1e3):,.0f} SNPs/s")
            ctx.close()
    # from storage: the dosages written to a file, then streamed through the
    # reader thread and three host buffers; page cache dropped for the file
    with tempfile.TemporaryDirectory(dir=os.environ.get("TMPDIR", "/tmp")) as d:
        for fmt, (H, _) in inputs.items():
            path = os.path.join(d, f"snps.{fmt}")
            H.numpy().tofile(path)
            for prec in ("fp64", "int8_emu"):
                ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=prec)
                fd = os.open(path, os.O_RDONLY)
                os.fsync(fd)
                os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
                os.close(fd)
                (_, _, _, _), fs = ctx.stream_file(path, m, torch.uint8 if fmt == "u8" else "u2")
                res[f"stream_file_{fmt}_{prec}"] = {
                    "snps_per_s": m / (fs.wall_ms / 1e3), "wall_ms": fs.wall_ms, "read_ms": fs.read_ms,
                    "file_GBps": fs.file_bytes / (fs.read_ms / 1e3) / 1e9 if fs.read_ms else None,
                    "compute_ms": fs.compute_ms, "note": "page cache of the file dropped before the run"}
                log(f"stream file {fmt} {prec}: {m / (fs.wall_ms / 1e3):,.0f} SNPs/s (read {fs.read_ms:.0f} ms)")
                ctx.close()
    del G_h, G2_h
    return res


def measure_scale(args, dev):
    """Streamed rate over a whole large study (m = 1,000,000 or 2,000,000): a
    pinned pool of distinct SNP blocks (about 21 GB) is streamed again and
    again until the study's m SNPs have gone through; the work per SNP is the
    same as for m distinct SNPs.  Setup excluded."""
    import torch

    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext

    w = synth.WORKLOADS[args.scale]
    # about 21 GB of pinned FP64, whole blocks: each pass restarts the copy pipeline, so passes are long
    pool = min(w.m, max(w.block_cols, int(21e9 / (8 * w.n)) // w.block_cols * w.block_cols))
    st = synth.make_study(w, m=pool)
    n, p, bc = w.n, w.p, w.block_cols
    host = torch.empty((pool, n), dtype=torch.float64).pin_memory()
    CH = 16384
    for j0 in range(0, pool, CH):
        j1 = min(pool, j0 + CH)
        host[j0:j1] = torch.from_numpy(synth.genotypes_u8(n, j0, j1, w.seed)).to(torch.float64)
    Phi_d, XL_d, y_d = (torch.tensor(np.ascontiguousarray(a), device=dev) for a in (st.Phi, st.XL, st.y))
    ctx = GLSContext(Phi_d, w.h2, XL_d, y_d, block_cols=bc)
    out = (torch.empty((pool, p), dtype=torch.float64).pin_memory(), torch.empty(pool, dtype=torch.float64).pin_memory(),
           torch.empty(pool, dtype=torch.float64).pin_memory(), torch.empty(pool, dtype=torch.int32).pin_memory())
    ctx.stream(host[:bc], out=tuple(o[:bc] for o in out))   # warm-up
    torch.cuda.synchronize()
    done, wall_ms, compute_ms, passes = 0, 0.0, 0.0, 0
    t0 = time.perf_counter()
    while done < w.m:
        k = min(pool, w.m - done)
        _, s_ = ctx.stream(host[:k], out=tuple(o[:k] for o in out))
        wall_ms += s_.wall_ms
        compute_ms += s_.compute_ms
        done += k
        passes += 1
    total = time.perf_counter() - t0
    ctx.close()
    res = {"workload": w.name, "n": n, "p": p, "m": w.m, "block_cols": bc, "pool_snps": pool, "passes": passes,
           "snps_per_s": w.m / total, "snps_per_s_device_wall": w.m / (wall_ms / 1e3), "compute_ms": compute_ms,
           "note": "PCIe-inclusive, setup excluded; a pinned pool of distinct SNPs streamed repeatedly"}
    log(f"scale {w.name}: {w.m:,} SNPs in {total:.2f} s -> {w.m / total:,.0f} SNPs/s ({passes} passes)")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1_n10k_m100k")
    ap.add_argument("--m", type=int, default=None, help="override the SNP count")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--sweeps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="SNPs the oracle solves for the CPU baseline (0: the whole study)")
    ap.add_argument("--no-stream", action="store_true", help="skip the streamed (pinned host memory) measurement")
    ap.add_argument("--no-forms", action="store_true", help="skip the mixed-precision and adjoint measurements")
    ap.add_argument("--no-bytes", action="store_true", help="skip the genotype-byte and packed-dosage measurements")
    ap.add_argument("--scale", default=None,
                    help="also stream a whole large workload (e.g. c2_n10k_m1M) from a cycled pinned pool")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM traffic counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; runs on several GPUs are not supported "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext, make_opts, workspace_bytes

    w = synth.WORKLOADS[args.workload]
    m = args.m or w.m
    n, p, bc, h2 = w.n, w.p, w.block_cols, w.h2
    dev = torch.device("cuda:0")
    log(f"workload {w.name}: n={n} p={p} m={m} block_cols={bc} h2={h2} precision={args.precision}")
    t = time.perf_counter()
    st = synth.make_study(w, m=m)
    log(f"study inputs generated in {time.perf_counter() - t:.1f}s")
    Phi_d = torch.tensor(st.Phi, device=dev)
    XL_d = torch.tensor(st.XL, device=dev)
    y_d = torch.tensor(st.y, device=dev)
    X_d = torch.empty((m, n), dtype=torch.float64, device=dev)
    CH = 16384
    t = time.perf_counter()
    for j0 in range(0, m, CH):
        j1 = min(m, j0 + CH)
        X_d[j0:j1] = torch.from_numpy(synth.genotypes_u8(n, j0, j1, w.seed)).to(dev).to(torch.float64)
    torch.cuda.synchronize()
    log(f"SNP matrix resident in HBM ({X_d.numel() * 8 / 1e9:.1f} GB) after {time.perf_counter() - t:.1f}s")

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy of 1 GiB done")

    b_d = torch.empty((m, p), dtype=torch.float64, device=dev)
    s2_d = torch.empty(m, dtype=torch.float64, device=dev)
    v_d = torch.empty(m, dtype=torch.float64, device=dev)
    st_d = torch.empty(m, dtype=torch.int32, device=dev)
    b_h = torch.empty((m, p), dtype=torch.float64).pin_memory()
    s2_h = torch.empty(m, dtype=torch.float64).pin_memory()
    v_h = torch.empty(m, dtype=torch.float64).pin_memory()
    st_h = torch.empty(m, dtype=torch.int32).pin_memory()
    phase_tot = {}

    def step(profile: bool):
        ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision,
                         refine_sweeps=args.sweeps)
        if profile:
            ctx.profile(True)
        for j0 in range(0, m, bc):
            j1 = min(m, j0 + bc)
            ctx.block_into(X_d[j0:j1], b_d[j0:j1], s2_d[j0:j1], v_d[j0:j1], st_d[j0:j1])
        b_h.copy_(b_d, non_blocking=True)
        s2_h.copy_(s2_d, non_blocking=True)
        v_h.copy_(v_d, non_blocking=True)
        st_h.copy_(st_d, non_blocking=True)
        if profile:
            for k, (cnt, ms) in ctx.profile_read().items():
                c0, m0 = phase_tot.get(k, (0, 0.0))
                phase_tot[k] = (c0 + cnt, m0 + ms)
        ctx.close()

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"timed step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = m / (ms_per_step / 1e3)
    log(f"{ms_per_step:.1f} ms/step -> {value:,.0f} SNPs/s")

    # setup-only time (excluded from nothing above; reported for context)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps).close()
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - ts) * 1e3

    wl, wms = phase_tot.get("whiten", (0, 0.0))
    flops_per_step = float(n) * n * m
    achieved = flops_per_step * args.steps / (wms / 1e3) / 1e12 if wms > 0 else None
    peak = PEAK_TFLOPS[args.precision]
    traffic = None
    if (args.precision == "fp64" and kernel_hash() == TRAFFIC_RECORD["kernel_sha1"] and n == TRAFFIC_RECORD["n"]
            and bc == TRAFFIC_RECORD["block_cols"]):
        traffic = TRAFFIC_RECORD["bytes_per_launch"]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": (achieved / peak) if achieved else None, "traffic": traffic,
                "traffic_unit": "bytes per full 8,192-SNP launch (HBM, rocprofv3 FETCH_SIZE+WRITE_SIZE, calibrated)",
                "kernel": "trmm_f64_dma_kernel (X~ = L^-1 X; 128 x 64 tiles, v_mfma_f64_4x4x4_4b_f64)",
                "launch_ms_avg": wms / wl if wl else None, "launches": wl,
                "flops_per_snp": float(n) * n}
    out = {
        "metric": METRIC, "value": value, "unit": "SNPs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else args.precision, "data": "synthetic",
        "config": {"workload": w.name, "n": n, "p": p, "m": m, "block_cols": bc, "h2": h2,
                   "precision": args.precision, "refine_sweeps": args.sweeps, "inputs": "HBM-resident"},
        "roofline": roofline,
        "phases_ms_per_step": {k: v[1] / args.steps for k, v in phase_tot.items()},
        "setup_ms": setup_ms,
        "snps_per_s_excl_setup": m / ((ms_per_step - setup_ms) / 1e3) if ms_per_step > setup_ms else None,
        "device_memory": {"peak_allocated_bytes": int(torch.cuda.max_memory_allocated()),
                          "workspace_bytes": workspace_bytes(n, p, make_opts(bc, args.precision, args.sweeps)),
                          "snp_matrix_bytes": int(X_d.numel() * 8)},
    }

    if not args.no_forms:
        out["forms"] = measure_forms(args, st, Phi_d, XL_d, y_d, X_d, m, dev)
    if not args.no_bytes:
        out["bytes"] = measure_bytes(args, st, Phi_d, XL_d, y_d, X_d, m, dev, b_h)
    if not args.no_stream:
        host = torch.empty((m, n), dtype=torch.float64).pin_memory()
        host.copy_(X_d)
        ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps)
        ctx.stream(host)
        torch.cuda.synchronize()
        (_, _, _, _), stats = ctx.stream(host)
        out["stream"] = {"snps_per_s": m / (stats.wall_ms / 1e3), "wall_ms": stats.wall_ms,
                         "compute_ms": stats.compute_ms, "h2d_GBps": stats.h2d_bytes / (stats.wall_ms / 1e3) / 1e9,
                         "blocks": stats.blocks, "note": "PCIe-inclusive: pinned host X_R, setup excluded"}
        ctx.close()
        ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps,
                         serial_stream=True)
        (_, _, _, _), ss = ctx.stream(host)
        out["stream"]["serial_snps_per_s"] = m / (ss.wall_ms / 1e3)
        out["stream"]["serial_wall_ms"] = ss.wall_ms
        ctx.close()
        del host
        log(f"streamed: {out['stream']['snps_per_s']:,.0f} SNPs/s")

    if args.scale:
        out["scale"] = measure_scale(args, dev)

    if not args.no_cpu_baseline:
        from oracle import gls_oracle as O
        S = m if args.cpu_sample <= 0 else min(args.cpu_sample, m)
        log(f"cpu baseline: oracle setup + {S} SNPs on the host, in blocks of {bc}")
        t = time.perf_counter()
        ost = O.Study(st.Phi, h2, st.XL, st.y)
        t_setup = time.perf_counter() - t
        g, gst = b_h.numpy(), st_h.numpy()
        t_blk, err, status_equal = 0.0, 0.0, True

        def check(j0, j1):
            nonlocal t_blk, err, status_equal
            XRs = st.snps(j0, j1)                  # drawing the inputs is not timed
            t = time.perf_counter()
            ref = ost.block(XRs.T)
            dt = time.perf_counter() - t
            ok = ref["status"] == 0
            e = np.max(np.abs(g[j0:j1][ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)
            err = max(err, float(e.max()) if e.size else 0.0)
            status_equal = status_equal and bool(np.array_equal(gst[j0:j1], ref["status"]))
            return dt

        for j0 in range(0, S, bc):
            t_blk += check(j0, min(S, j0 + bc))
        if S < m:
            check(m - 64, m)                        # and the study's ragged tail
        cpu_total = t_setup + (m / S) * t_blk
        whole = "the whole study" if S == m else "whole-study time extrapolated linearly in m"
        out["cpu_baseline"] = {"value": m / cpu_total, "unit": "SNPs/s", "cores": blas_threads(), "kind": "oracle",
                               "sample": f"oracle setup (Cholesky of M, covariate terms) {t_setup:.1f}s + SNPs "
                                         f"[0,{S}) in blocks of {bc} {t_blk:.1f}s; {whole}",
                               "host": host_info()}
        # parity of this run's outputs against the oracle on the same SNPs
        out["parity_vs_oracle"] = {"snps": int(S + (64 if S < m else 0)), "max_rel_err_b": err,
                                   "status_equal": status_equal}
        log(f"cpu baseline {out['cpu_baseline']['value']:,.0f} SNPs/s; max rel err of b over {S} SNPs {err:.2e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
