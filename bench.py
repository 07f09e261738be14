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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def blas_threads() -> int:
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n = [d.get("num_threads", 0) for d in info if d.get("user_api") == "blas"]
        return int(max(n)) if n else (os.cpu_count() or 1)
    except Exception:
        return os.cpu_count() or 1


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
    ap.add_argument("--cpu-sample", type=int, default=8192, help="SNPs the oracle solves for the CPU baseline")
    ap.add_argument("--stream", action="store_true", help="also time the streamed path from pinned host memory")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not part of this build "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1302_4332_amd import synth
    from paper_1302_4332_amd.gls import GLSContext

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
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": (achieved / peak) if achieved else None, "traffic": None,
                "kernel": "gemm_f64_kernel<64,64,16,1,4,false,false,MAP_XCD,VEC,M4> (X~ = L^-1 X)",
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
    }

    if args.stream:
        host = torch.empty((m, n), dtype=torch.float64).pin_memory()
        host.copy_(X_d)
        ctx = GLSContext(Phi_d, h2, XL_d, y_d, block_cols=bc, precision=args.precision, refine_sweeps=args.sweeps)
        ctx.stream(host)
        torch.cuda.synchronize()
        (_, _, _, _), stats = ctx.stream(host)
        out["stream"] = {"snps_per_s": m / (stats.wall_ms / 1e3), "wall_ms": stats.wall_ms,
                         "compute_ms": stats.compute_ms, "h2d_GBps": stats.h2d_bytes / (stats.wall_ms / 1e3) / 1e9,
                         "blocks": stats.blocks}
        ctx.close()
        del host
        log(f"streamed: {out['stream']['snps_per_s']:,.0f} SNPs/s")

    if not args.no_cpu_baseline:
        from oracle import gls_oracle as O
        S = min(args.cpu_sample, m)
        log(f"cpu baseline: oracle setup + {S} SNPs on the host")
        t = time.perf_counter()
        ost = O.Study(st.Phi, h2, st.XL, st.y)
        t_setup = time.perf_counter() - t
        XRs = st.snps(0, S)
        t = time.perf_counter()
        ref = ost.block(XRs.T)
        t_blk = time.perf_counter() - t
        cpu_total = t_setup + (m / S) * t_blk
        out["cpu_baseline"] = {"value": m / cpu_total, "unit": "SNPs/s", "cores": blas_threads(), "kind": "oracle",
                               "sample": f"oracle setup (Cholesky of M, covariate terms) {t_setup:.1f}s + SNPs "
                                         f"[0,{S}) {t_blk:.1f}s, whole-study time extrapolated linearly in m"}
        # sampled parity of this run's outputs (first block and the ragged tail)
        tail = st.snps(m - 64, m)
        ref_t = ost.block(tail.T)
        g = b_h.numpy()
        ok = ref["status"] == 0
        e1 = np.max(np.abs(g[:S][ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)
        e2 = np.max(np.abs(g[m - 64:] - ref_t["b"]), axis=1) / np.max(np.abs(ref_t["b"]), axis=1)
        out["parity_sampled"] = {"snps": int(S + 64), "max_rel_err_b": float(max(e1.max(), e2.max())),
                                 "status_equal": bool(np.array_equal(st_h.numpy()[:S], ref["status"]))}
        log(f"cpu baseline {out['cpu_baseline']['value']:,.0f} SNPs/s; sampled max rel err "
            f"{out['parity_sampled']['max_rel_err_b']:.2e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
