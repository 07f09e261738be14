#!/usr/bin/env python3
"""Throughput of the streamed GWAS GLS hot path on one MI355X.

One step = one whole study streamed from page-locked host memory (the
paper's setting, Sec. 3.1): every SNP block copied to the device through the
double-buffered pipeline, the triangular product, the per-SNP products and
p x p solves, and the results copied back into host arrays, from the first
copy to the last result landed.  The setup (M, Cholesky, inverse factor,
covariate terms) runs once before the steps and is reported separately
(setup_ms), as the paper times it apart.  The value is m over the median
step time.  The whole study with the SNP matrix resident in HBM, setup
included, is reported as hbm_resident.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c1_n10k_m100k]
"""
from __future__ import annotations

import argparse
import dataclasses
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
TRAFFIC_RECORD = {"kernel_sha1": "eba3c7d612aaf075", "n": 10000, "block_cols": 8192, "bytes_per_launch": 28.49e9}


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


def timed_runs(fn, reps):
    """Time fn() reps times (each bracketed by device synchronizations);
    returns (median ms, every run's ms, the value fn returned on the median run)."""
    import torch

    runs = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        runs.append(((time.perf_counter() - t0) * 1e3, out))
    order = sorted(range(reps), key=lambda i: runs[i][0])
    med = runs[order[reps // 2]]
    return med[0], [r[0] for r in runs], med[1]


def measure_forms(args, st, Phi_d, XL_d, y_d, X_d, m, dev):
    """Mixed-precision forms on the same workload, and the adjoint on the
    n = 4,096 differentiation study; the median of args.sub_reps timed studies
    each (after one untimed)."""
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
        ms, runs, ph = timed_runs(lambda: study(True), args.sub_reps)
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
            "phases_ms": {k: v[1] for k, v in ph.items()}, "runs_ms": runs}
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
        ms, runs, gh = timed_runs(fwd_bwd, args.sub_reps)
        res[f"adjoint_c3_{prec}"] = {"workload": w3.name, "ms_fwd_bwd": ms, "snps_per_s": w3.m / (ms / 1e3),
                                     "h2_grad": float(gh), "runs_ms": runs}
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
    ms, runs, ph = timed_runs(lambda: study(True), args.sub_reps)
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
        "max_rel_diff_vs_fp64_path": float(rel.max()), "runs_ms": runs,
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
            stats = sorted((ctx.stream(H, packed=packed)[1] for _ in range(args.sub_reps)), key=lambda x: x.wall_ms)
            ss = stats[len(stats) // 2]
            res[f"stream_{fmt}_{prec}"] = {"snps_per_s": m / (ss.wall_ms / 1e3), "wall_ms": ss.wall_ms,
                                           "compute_ms": ss.compute_ms,
                                           "h2d_GBps": ss.h2d_bytes / (ss.wall_ms / 1e3) / 1e9,
                                           "runs_wall_ms": [x.wall_ms for x in stats]}
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
                stats = []
                for _ in range(args.sub_reps):
                    fd = os.open(path, os.O_RDONLY)
                    os.fsync(fd)
                    os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
                    os.close(fd)
                    stats.append(ctx.stream_file(path, m, torch.uint8 if fmt == "u8" else "u2")[1])
                stats.sort(key=lambda x: x.wall_ms)
                fs = stats[len(stats) // 2]
                res[f"stream_file_{fmt}_{prec}"] = {
                    "snps_per_s": m / (fs.wall_ms / 1e3), "wall_ms": fs.wall_ms, "read_ms": fs.read_ms,
                    "file_GBps": fs.file_bytes / (fs.read_ms / 1e3) / 1e9 if fs.read_ms else None,
                    "compute_ms": fs.compute_ms, "runs_wall_ms": [x.wall_ms for x in stats],
                    "note": "page cache of the file dropped before each run"}
                log(f"stream file {fmt} {prec}: {m / (fs.wall_ms / 1e3):,.0f} SNPs/s (read {fs.read_ms:.0f} ms)")
                ctx.close()
    del G_h, G2_h
    return res


def measure_scale(args, dev):
    """Streamed rate over a whole large study (m = 1,000,000 or 2,000,000) in
    the precision --precision / --sweeps name: a pinned pool of distinct SNP
    blocks (about 21 GB) is streamed untimed until two passes agree, then again
    and again until the study's m SNPs have gone through; the work per SNP is
    the same as for m distinct SNPs.  Setup excluded.  For a refined precision
    the last pass's b is compared with plain FP64 on the same SNPs."""
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
    ctx = GLSContext(Phi_d, w.h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps)
    out = (torch.empty((pool, p), dtype=torch.float64).pin_memory(), torch.empty(pool, dtype=torch.float64).pin_memory(),
           torch.empty(pool, dtype=torch.float64).pin_memory(), torch.empty(pool, dtype=torch.int32).pin_memory())
    # warm-up: whole passes over the pool until two in a row agree within 3% in solve time (at most four; after
    # the host-side fill the first passes of a run solved 15-30% slower on some boxes)
    prev = None
    for _ in range(4):
        cms = ctx.stream(host, out=out)[1].compute_ms
        if prev is not None and abs(cms - prev) <= 0.03 * prev:
            break
        prev = cms
    torch.cuda.synchronize()
    done, wall_ms, compute_ms, passes = 0, 0.0, 0.0, 0
    pass_ms = []   # (device wall, summed solve time) per pass: the copies hide under the solves when they agree
    t0 = time.perf_counter()
    while done < w.m:
        k = min(pool, w.m - done)
        _, s_ = ctx.stream(host[:k], out=tuple(o[:k] for o in out))
        wall_ms += s_.wall_ms
        compute_ms += s_.compute_ms
        pass_ms.append((round(s_.wall_ms, 1), round(s_.compute_ms, 1)))
        done += k
        passes += 1
    total = time.perf_counter() - t0
    ctx.close()
    err_vs_fp64 = None
    if args.precision != "fp64":   # the pool's last outputs against plain FP64 on the same SNPs
        k = min(pool, w.m - (passes - 1) * pool)
        ref_ctx = GLSContext(Phi_d, w.h2, XL_d, y_d, block_cols=bc)
        (rb, _, _, rst), _ = ref_ctx.stream(host[:k])
        ref_ctx.close()
        ok = (rst.numpy() == 0) & (out[3][:k].numpy() == 0)
        rb, gb = rb.numpy()[ok], out[0][:k].numpy()[ok]
        err_vs_fp64 = float(np.max(np.max(np.abs(gb - rb), axis=1) / np.max(np.abs(rb), axis=1)))
        log(f"scale {w.name} {args.precision} x{args.sweeps}: max rel err of b against FP64 {err_vs_fp64:.2e} "
            f"over {int(ok.sum()):,} SNPs")
    res = {"workload": w.name, "n": n, "p": p, "m": w.m, "block_cols": bc, "pool_snps": pool, "passes": passes,
           "precision": args.precision, "refine_sweeps": args.sweeps, "max_rel_err_b_vs_fp64": err_vs_fp64,
           "snps_per_s": w.m / total, "snps_per_s_device_wall": w.m / (wall_ms / 1e3), "compute_ms": compute_ms,
           "pass_wall_compute_ms": pass_ms,
           "note": "PCIe-inclusive, setup excluded; a pinned pool of distinct SNPs streamed repeatedly"}
    log(f"scale {w.name}: {w.m:,} SNPs in {total:.2f} s -> {w.m / total:,.0f} SNPs/s ({passes} passes)")
    return res


def measure_gemm_ceiling(dev):
    """The vendor library's dense products (torch.matmul, which calls hipBLASLt or
    rocBLAS) on contiguous operands at the per-block shape M = K = 10,240,
    N = 8,192: a measured ceiling for each matrix-core precision beside the
    datasheet peak.  Measurement only; no product of the solver goes through it."""
    import torch

    M, N, K = 10240, 8192, 10240
    res = {"shape_mnk": [M, N, K], "library": "torch.matmul (hipBLASLt / rocBLAS)"}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32), ("fp16", torch.float16),
                     ("bf16", torch.bfloat16)):
        g = torch.Generator(device=dev).manual_seed(5)
        A = torch.rand((M, K), device=dev, dtype=dt, generator=g)
        B = torch.rand((K, N), device=dev, dtype=dt, generator=g)
        C = torch.matmul(A, B)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            torch.matmul(A, B, out=C)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * M * N * K / (ms / 1e3) / 1e12
        peak = PEAK_TFLOPS[{"fp64": "fp64", "fp32": "fp32_ir", "fp16": "fp16_ir", "bf16": "bf16_ir"}[name]]
        res[name] = {"ms": ms, "tflops": tf, "peak": peak, "frac": tf / peak}
        log(f"vendor dense {name} product {M}x{N}x{K}: {ms:.2f} ms, {tf:.1f} TFLOP/s ({tf / peak:.2f} of peak)")
        del A, B, C
    return res


def measure_scale_grad(args, dev):
    """d loss / d h2 and d loss / d y of the loss sum_i t_i^2 over a whole large
    study whose SNPs stay in host memory (m = 2,000,000 at n = 20,000): per pass
    over a pinned pool of distinct SNP blocks (about 21 GB), the forward stream
    (gls_stream), the loss's cotangents on the device, and the streamed adjoint
    (gls_stream_backward); after m SNPs, gls_backward_finish.  Setup included;
    peak device memory recorded."""
    import torch

    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext, t2_loss

    w = synth.WORKLOADS[args.scale_grad]
    if args.grad_m:
        w = dataclasses.replace(w, m=args.grad_m)
    n, p, bc = w.n, w.p, w.block_cols
    pool = min(w.m, max(bc, int(21e9 / (8 * n)) // bc * bc))
    st = synth.make_study(w, m=pool)
    host = torch.empty((pool, n), dtype=torch.float64).pin_memory()
    CH = 16384
    for j0 in range(0, pool, CH):
        j1 = min(pool, j0 + CH)
        host[j0:j1] = torch.from_numpy(synth.genotypes_u8(n, j0, j1, w.seed)).to(torch.float64)
    Phi_d, XL_d, y_d = (torch.tensor(np.ascontiguousarray(a), device=dev) for a in (st.Phi, st.XL, st.y))
    pin = lambda *shape: torch.empty(shape, dtype=torch.float64).pin_memory()
    out = (pin(pool, p), pin(pool), pin(pool), torch.empty(pool, dtype=torch.int32).pin_memory())
    cot = (pin(pool, p), pin(pool), pin(pool))
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    ctx = GLSContext(Phi_d, w.h2, XL_d, y_d, block_cols=bc, precision=args.grad_precision,
                     refine_sweeps=args.grad_sweeps, keep_for_grad=True)
    done, loss, fwd_ms, bwd_ms, passes = 0, 0.0, 0.0, 0.0, []
    while done < w.m:
        k = min(pool, w.m - done)
        tp = time.perf_counter()
        _, sf = ctx.stream(host[:k], out=tuple(o[:k] for o in out))
        leaves = [o[:k].to(dev).requires_grad_(True) for o in out[:3]]
        value = t2_loss(*leaves)
        for c, g in zip(cot, torch.autograd.grad(value, leaves)):
            c[:k].copy_(g)
        loss += float(value.detach())
        sb = ctx.stream_backward(host[:k], *(c[:k] for c in cot))
        fwd_ms += sf.wall_ms
        bwd_ms += sb.wall_ms
        done += k
        passes.append({"snps": k, "ms": round((time.perf_counter() - tp) * 1e3, 1), "forward_wall_ms": round(sf.wall_ms, 1),
                       "backward_wall_ms": round(sb.wall_ms, 1), "backward_compute_ms": round(sb.compute_ms, 1)})
        log(f"grad pass {len(passes)}: {done:,} of {w.m:,} SNPs, forward {sf.wall_ms:.0f} ms, "
            f"backward {sb.wall_ms:.0f} ms")
    y_grad, h2_grad = ctx.backward_finish()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ctx.close()
    peak = int(torch.cuda.max_memory_allocated())
    mem = int(torch.cuda.get_device_properties(0).total_memory)
    res = {"workload": w.name, "n": n, "p": p, "m": w.m, "block_cols": bc, "precision": args.grad_precision,
           "refine_sweeps": args.grad_sweeps, "pool_snps": pool, "loss": loss, "h2_grad": float(h2_grad),
           "y_grad_norm": float(torch.linalg.norm(y_grad)), "seconds": total, "snps_per_s": w.m / total,
           "forward_wall_ms": fwd_ms, "backward_wall_ms": bwd_ms, "passes": passes,
           "peak_device_bytes": peak, "device_bytes": mem, "peak_fraction": peak / mem,
           "note": "setup, forward stream, loss cotangents, streamed adjoint and finish; a pinned pool of distinct "
                   "SNPs streamed repeatedly"}
    log(f"scale grad {w.name}: {w.m:,} SNPs forward + backward in {total:.1f} s, d loss/d h2 {float(h2_grad):.6e}, "
        f"peak device memory {peak / 1e9:.1f} GB ({peak / mem:.1%})")
    return res


def measure_resident(args, Phi_d, XL_d, y_d, X_d, m, n, p, bc, h2, steps):
    """The whole study with the SNP matrix already in HBM, setup included:
    setup, every block, results copied to host memory."""
    import torch

    from paper_1302_4332_amd.gls import GLSContext

    dev = X_d.device
    b_d = torch.empty((m, p), dtype=torch.float64, device=dev)
    s2_d = torch.empty(m, dtype=torch.float64, device=dev)
    v_d = torch.empty(m, dtype=torch.float64, device=dev)
    st_d = torch.empty(m, dtype=torch.int32, device=dev)
    b_h = torch.empty((m, p), dtype=torch.float64).pin_memory()

    def study():
        ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps)
        for j0 in range(0, m, bc):
            j1 = min(m, j0 + bc)
            ctx.block_into(X_d[j0:j1], b_d[j0:j1], s2_d[j0:j1], v_d[j0:j1], st_d[j0:j1])
        b_h.copy_(b_d, non_blocking=True)
        ctx.close()

    study()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        study()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    log(f"HBM-resident whole study incl. setup: {ms:.1f} ms -> {m / (ms / 1e3):,.0f} SNPs/s")
    return {"snps_per_s": m / (ms / 1e3), "ms_per_study": ms, "studies": steps,
            "note": "SNP matrix resident in HBM; setup, every block and the results' copy to host timed"}


def cpu_baselines(args, st, m, bc, h2, g_b, g_status):
    """The oracle on the host: the whole study on every BLAS thread (or a
    sample, --cpu-sample), and a bounded sample on one thread; both check this
    run's streamed outputs on the SNPs they solve."""
    from oracle import gls_oracle as O

    S = m if args.cpu_sample <= 0 else min(args.cpu_sample, m)
    log(f"cpu baseline: oracle setup + {S} SNPs on the host, in blocks of {bc}")
    t = time.perf_counter()
    ost = O.Study(st.Phi, h2, st.XL, st.y)
    t_setup = time.perf_counter() - t
    t_blk, err, status_equal = 0.0, 0.0, True

    def check(j0, j1, study):
        nonlocal err, status_equal
        XRs = st.snps(j0, j1)                  # drawing the inputs is not timed
        t = time.perf_counter()
        ref = study.block(XRs.T)
        dt = time.perf_counter() - t
        ok = ref["status"] == 0
        e = np.max(np.abs(g_b[j0:j1][ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)
        err = max(err, float(e.max()) if e.size else 0.0)
        status_equal = status_equal and bool(np.array_equal(g_status[j0:j1], ref["status"]))
        return dt

    for j0 in range(0, S, bc):
        t_blk += check(j0, min(S, j0 + bc), ost)
    if S < m:
        check(m - 64, m, ost)                   # and the study's ragged tail
    cpu_total = t_setup + (m / S) * t_blk
    whole = "the whole study" if S == m else "whole-study time extrapolated linearly in m"
    res = {"value": m / cpu_total, "unit": "SNPs/s", "cores": blas_threads(), "kind": "oracle",
           "sample": f"oracle setup (Cholesky of M, covariate terms) {t_setup:.1f}s + SNPs "
                     f"[0,{S}) in blocks of {bc} {t_blk:.1f}s; {whole}",
           "host": host_info()}
    parity = {"snps": int(S + (64 if S < m else 0)), "max_rel_err_b": err, "status_equal": status_equal,
              "outputs": "the streamed outputs of the last timed step"}
    log(f"cpu baseline {res['value']:,.0f} SNPs/s; max rel err of b over {S} SNPs {err:.2e}")
    if args.cpu_single_sample > 0:
        import threadpoolctl
        S1 = min(args.cpu_single_sample, m)
        with threadpoolctl.threadpool_limits(1):
            t = time.perf_counter()
            ost1 = O.Study(st.Phi, h2, st.XL, st.y)
            t1_setup = time.perf_counter() - t
            t1_blk = check(0, S1, ost1)
        total1 = t1_setup + (m / S1) * t1_blk
        res["single_thread"] = {"value": m / total1, "unit": "SNPs/s", "cores": 1,
                                "sample": f"oracle setup {t1_setup:.1f}s + SNPs [0,{S1}) {t1_blk:.1f}s on one "
                                          f"thread; whole-study time extrapolated linearly in m"}
        log(f"cpu baseline, one thread: {m / total1:,.0f} SNPs/s")
    return res, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1_n10k_m100k")
    ap.add_argument("--m", type=int, default=None, help="override the SNP count")
    ap.add_argument("--n", type=int, default=None, help="override the sample count (e.g. 10007: n not a multiple "
                    "of the product's k step)")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--sweeps", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="SNPs the oracle solves for the CPU baseline (0: the whole study)")
    ap.add_argument("--cpu-single-sample", type=int, default=2048,
                    help="SNPs the one-thread oracle run solves (0: skip it)")
    ap.add_argument("--resident-steps", type=int, default=2,
                    help="whole studies timed with the SNP matrix resident in HBM (0: skip)")
    ap.add_argument("--no-serial", action="store_true", help="skip the no-overlap ablation")
    ap.add_argument("--no-forms", action="store_true", help="skip the mixed-precision and adjoint measurements")
    ap.add_argument("--no-bytes", action="store_true", help="skip the genotype-byte and packed-dosage measurements")
    ap.add_argument("--sub-reps", type=int, default=3,
                    help="timed runs of each forms / bytes / adjoint measurement (the median is reported)")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the vendor-library dense product ceilings")
    ap.add_argument("--scale", default=None,
                    help="also stream a whole large workload (e.g. c2_n10k_m1M) from a cycled pinned pool")
    ap.add_argument("--scale-grad", default=None,
                    help="also compute d loss / d h2 over a whole large streamed workload (e.g. c4_n20k_p8)")
    ap.add_argument("--grad-precision", default="fp32_ir", help="precision of the --scale-grad study")
    ap.add_argument("--grad-sweeps", type=int, default=2, help="refinement sweeps of the --scale-grad study")
    ap.add_argument("--grad-m", type=int, default=None, help="override the SNP count of the --scale-grad study")
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
    if args.n:
        w = dataclasses.replace(w, n=args.n, name=f"{w.name}_n{args.n}")
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
    host = torch.empty((m, n), dtype=torch.float64).pin_memory()
    CH = 16384
    t = time.perf_counter()
    for j0 in range(0, m, CH):
        j1 = min(m, j0 + CH)
        host[j0:j1] = torch.from_numpy(synth.genotypes_u8(n, j0, j1, w.seed)).to(torch.float64)
    log(f"SNP matrix in page-locked host memory ({host.numel() * 8 / 1e9:.1f} GB) after {time.perf_counter() - t:.1f}s")

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy of 1 GiB done")

    # setup alone (M, Cholesky, inverse factor, covariate terms): median of three
    setups = []
    for _ in range(3):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps).close()
        torch.cuda.synchronize()
        setups.append((time.perf_counter() - ts) * 1e3)
    setup_ms = float(np.median(setups))
    log(f"setup {setup_ms:.1f} ms (median of 3)")

    # the headline: the study streamed from page-locked host memory through the
    # double-buffered pipeline, first copy to last result in host memory
    ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps)
    out_h = (torch.empty((m, p), dtype=torch.float64).pin_memory(), torch.empty(m, dtype=torch.float64).pin_memory(),
             torch.empty(m, dtype=torch.float64).pin_memory(), torch.empty(m, dtype=torch.int32).pin_memory())
    for i in range(args.warmup):
        ctx.stream(host, out=out_h)
        log(f"warmup step {i + 1}/{args.warmup} done")
    ctx.profile(True)
    ctx.profile_read(reset=True)
    step_ms, dev_wall, h2d = [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        _, stats = ctx.stream(host, out=out_h)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        dev_wall.append(stats.wall_ms)
        h2d += stats.h2d_bytes
        log(f"timed step {i + 1}/{args.steps}: {step_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = ctx.profile_read(reset=True)
    blocks = stats.blocks
    ctx.close()
    mean_ms = (t1 - t0) * 1e3 / args.steps
    med_ms = float(np.median(step_ms))
    value = m / (med_ms / 1e3)
    log(f"streamed: median {med_ms:.1f} ms/step -> {value:,.0f} SNPs/s (mean {mean_ms:.1f} ms)")

    wl, wms = phases["whiten"]
    flops = float(n) * n * m * args.steps
    achieved = flops / (wms / 1e3) / 1e12 if wms > 0 else None
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
                "flops_per_snp": float(n) * n,
                "timing": "HIP events around each launch on the compute stream, over the timed streamed steps"}
    out = {
        "metric": METRIC, "value": value, "unit": "SNPs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": med_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else args.precision, "data": "synthetic",
        "config": {"workload": w.name, "n": n, "p": p, "m": m, "block_cols": bc, "h2": h2,
                   "precision": args.precision, "refine_sweeps": args.sweeps,
                   "inputs": "pinned-host, streamed", "setup": "excluded (reported as setup_ms)"},
        "roofline": roofline,
        "step_ms": step_ms, "ms_per_step_mean": mean_ms, "step_statistic": "median",
        "device_wall_ms": dev_wall, "h2d_GBps": h2d / (sum(step_ms) / 1e3) / 1e9, "stream_blocks": blocks,
        "phases_ms_per_step": {k: v[1] / args.steps for k, v in phases.items()},
        "setup_ms": setup_ms, "setup_ms_samples": setups,
        "snps_per_s_incl_setup": m / ((med_ms + setup_ms) / 1e3),
        "device_memory": {"peak_allocated_bytes": int(torch.cuda.max_memory_allocated()),
                          "workspace_bytes": workspace_bytes(n, p, make_opts(bc, args.precision, args.sweeps))},
    }
    if not args.no_serial:
        sctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps,
                          serial_stream=True)
        _, ss = sctx.stream(host)
        sctx.close()
        out["serial_stream"] = {"snps_per_s": m / (ss.wall_ms / 1e3), "wall_ms": ss.wall_ms,
                                "note": "no-overlap ablation: copy, solve and results one after another"}
        log(f"serial stream: {m / (ss.wall_ms / 1e3):,.0f} SNPs/s")

    need_resident = args.resident_steps > 0 or not args.no_forms or not args.no_bytes
    X_d = None
    if need_resident:
        X_d = host.to(dev)
        if args.resident_steps > 0:
            out["hbm_resident"] = measure_resident(args, Phi_d, XL_d, y_d, X_d, m, n, p, bc, h2, args.resident_steps)
    if not args.no_forms:
        out["forms"] = measure_forms(args, st, Phi_d, XL_d, y_d, X_d, m, dev)
    if not args.no_bytes:
        out["bytes"] = measure_bytes(args, st, Phi_d, XL_d, y_d, X_d, m, dev, out_h[0])
    del X_d
    if not args.no_ceiling:
        out["gemm_ceiling"] = measure_gemm_ceiling(dev)
    if args.scale:
        out["scale"] = measure_scale(args, dev)
    if args.scale_grad:
        out["scale_grad"] = measure_scale_grad(args, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity_vs_oracle"] = cpu_baselines(args, st, m, bc, h2, out_h[0].numpy(),
                                                                     out_h[3].numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
