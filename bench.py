#!/usr/bin/env python3
"""Benchmark of the scatter-accumulate reverse-mode path on one MI355X.

A step is one GMM gradient evaluation (dex_fwd + dex_vjp: F and the cotangents
of alphas, means, qd and l) at N=100000, D=64, K=200 with BF16 matrix-core
products and FP32 accumulation, inputs resident in HBM. Prints one JSON line.

The line also carries, measured in the same run:
  roofline      the dominant kernel's algorithmic FLOP rate against the BF16
                dense peak, its duration taken live with HIP events;
  fp32_form     the same gradient with FP32 matrix-core products;
  rows          the other workloads of the path (gather / scatter-accumulate,
                histogram, batched GMM, checkpointed stencil adjoint), each with
                its kernel time and roofline fraction;
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample, and the
                GPU result's error against it on that sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GMM grad evals/s (N=1e5,D=64,K=200) + bwd/fwd ratio + HBM/MFMA roofline %"
PEAK = {"bf16": 2500.0, "fp32": 157.3, "hbm": 8000.0}  # TFLOP/s, TFLOP/s, GB/s
KERNEL_SOURCES = {
    "gmm_vjp": ["gmm_dev.h", "gmm_mfma_inst.hip", "gmm_host.h"],
    "gmm_fwd": ["gmm_dev.h", "gmm_mfma_inst.hip", "gmm_host.h", "gmm_qf.h"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2104_05372_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != src_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return rec.get("bytes_per_launch")


def timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


# ---------------------------------------------------------------------------
def gmm_setup(torch, dex, g, variant, dev, configs=None):
    t = [torch.tensor(a, device=dev) for a in (g.alphas, g.means, g.qd, g.l, g.x)]
    d = dex.gmm_desc(g.N, g.D, g.K, dex.DEX_F32, variant)
    F = torch.empty(1, device=dev)
    f = torch.empty(g.N, device=dev)
    cache = torch.empty(dex.dex_workspace_bytes(d, dex.DEX_WS_RESID), dtype=torch.uint8, device=dev)
    wsf = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev)
    wsb = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_VJP), dev)
    ct = torch.ones(1, device=dev)
    grads = [torch.empty_like(x) for x in t[:4]]
    if configs:
        bf, bb = configs
    else:
        bf = dex.dex_autotune(d, dex.DEX_WS_FWD, t, [F], [f, cache], [], [], wsf)
        dex.dex_fwd(d, t, [F], [f, cache], wsf)
        bb = dex.dex_autotune(d, dex.DEX_WS_VJP, t, [], [f, cache], [ct], grads, wsb)
    dfw = dex.gmm_desc(g.N, g.D, g.K, dex.DEX_F32, variant, bf)
    dbw = dex.gmm_desc(g.N, g.D, g.K, dex.DEX_F32, variant, bb)

    def fwd():
        dex.dex_fwd(dfw, t, [F], [f, cache], wsf)

    def vjp():
        dex.dex_vjp(dbw, t, [f, cache], [ct], grads, 0, wsb)

    return dict(t=t, d=d, F=F, grads=grads, fwd=fwd, vjp=vjp, cfg=(bf, bb))


def run_headline(torch, dex, workloads, args, dev):
    g = workloads.gmm_large()
    N, D, K = g.N, g.D, g.K
    variant = {"bf16": dex.DEX_GMM_BF16, "bf16x3": dex.DEX_GMM_BF16X3, "fp32": dex.DEX_GMM_PLAIN}[args.variant]
    cfgs = tuple(int(v) for v in args.configs.split(",")) if args.configs else None
    S = gmm_setup(torch, dex, g, variant, dev, cfgs)
    sync = torch.cuda.synchronize

    def step():
        S["fwd"]()
        S["vjp"]()

    for _ in range(args.warmup):
        step()
    sync()
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    sync()
    t0 = time.perf_counter()
    for e in ev:
        e[0].record()
        S["fwd"]()
        e[1].record()
        S["vjp"]()
        e[2].record()
    sync()
    elapsed = time.perf_counter() - t0
    dex.dex_profile_enable(False)
    fwd_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / len(ev)
    vjp_ms = sum(b.elapsed_time(c) for _, b, c in ev) / len(ev)
    kf_ms, kf_n = dex.dex_profile_read("GMM_FWD")
    kb_ms, kb_n = dex.dex_profile_read("GMM_VJP")
    tri = D * (D + 1) * N * K        # forward: y = Q r, triangular, 2 flops per multiply-add
    mom = D * (D + 3) * N * K        # reverse: symmetric sum of w x x^T (D(D+1)/2 entries) and w x
    kern = {
        "gmm_fwd": {"avg_ms": kf_ms / max(kf_n, 1), "flop_per_launch": tri},
        "gmm_vjp": {"avg_ms": kb_ms / max(kb_n, 1), "flop_per_launch": mom},
    }
    for k in kern.values():
        k["tflops"] = k["flop_per_launch"] / (k["avg_ms"] * 1e-3) / 1e12
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    peak = PEAK["fp32"] if args.variant == "fp32" else PEAK["bf16"]
    roof = {"bound": "mfma", "kernel": dom, "achieved": round(kern[dom]["tflops"], 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(kern[dom]["tflops"] / peak, 4),
            "traffic": traffic_from_profiles(dom),
            "kernels": {k: {"avg_ms": round(v["avg_ms"], 4), "tflops": round(v["tflops"], 2),
                            "frac": round(v["tflops"] / peak, 4)} for k, v in kern.items()},
            "flop_count": "forward D(D+1)NK (triangular y = Q r); reverse D(D+3)NK (symmetric "
                          "weighted moment sum_i w x x^T and sum_i w x per component)"}
    res = dict(value=args.steps / elapsed, ms=elapsed / args.steps * 1e3, fwd_ms=fwd_ms, vjp_ms=vjp_ms,
               roofline=roof, cfg=S["cfg"], g=g, S=S)
    return res


def run_fp32_form(torch, dex, g, dev, steps):
    S = gmm_setup(torch, dex, g, dex.DEX_GMM_PLAIN, dev)
    for _ in range(2):
        S["fwd"]()
        S["vjp"]()
    ms = timed(lambda: (S["fwd"](), S["vjp"]()), steps, torch.cuda.synchronize) * 1e3
    fl = (g.D * (g.D + 1) + g.D * (g.D + 3)) * g.N * g.K
    return {"grad_evals_per_s": round(1e3 / ms, 2), "ms_per_step": round(ms, 3),
            "tflops": round(fl / (ms * 1e-3) / 1e12, 2),
            "frac_fp32_peak": round(fl / (ms * 1e-3) / 1e12 / PEAK["fp32"], 4),
            "config": list(S["cfg"])}


# ---------------------------------------------------------------------------
def row_scatter(torch, dex, workloads, dev, steps, scatter_config=1):
    import numpy as np
    c = workloads.SCATTER
    V, R, n = c["rows"], c["row_len"], c["n"]
    gen = torch.Generator(device=dev).manual_seed(c["seed"])
    idx_np = workloads.zipf_table_indices(n, V, c["s"], c["seed"])
    touched = int(np.unique(idx_np).size)
    T = torch.randn(V, R, device=dev, generator=gen)
    idx = torch.tensor(idx_np, device=dev)
    w = torch.rand(n, device=dev, generator=gen) * 2 - 1
    g = torch.randn(n, R, device=dev, generator=gen)
    out = torch.empty(n, R, device=dev)
    dT = torch.empty_like(T)
    dw = torch.empty_like(w)
    d = dex.gather_desc(V, R, n)
    wsb = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_VJP), dev)
    dv = dex.gather_desc(V, R, n)
    dv.config = scatter_config

    def fwd():
        dex.dex_fwd(d, [T, idx, w], [out], [])

    def vjp():
        dex.dex_vjp(dv, [T, idx, w], [], [g], [dT, dw], 0, wsb)

    # forward mode: dT (filled by the reverse pass) and w serve as the tangents
    # of T and w, out receives the tangent of the output
    def jvp():
        dex.dex_jvp(d, [T, idx, w], [dT, w], [out])

    fwd()
    vjp()
    torch.cuda.synchronize()
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    f_ms = timed(fwd, steps, torch.cuda.synchronize) * 1e3
    b_ms = timed(vjp, steps, torch.cuda.synchronize) * 1e3
    j_ms = timed(jvp, steps, torch.cuda.synchronize) * 1e3 if scatter_config == 1 else None
    dex.dex_profile_enable(False)
    res = {"workload": f"gather/scatter table {V}x{R} f32, {n} Zipf(1.1) indices",
           "scatter_form": {1: "block sort + run sums + atomics", 2: "radix sort, fixed-order run sums"}[
               scatter_config],
           "fwd_ms": round(f_ms, 4), "vjp_ms": round(b_ms, 4), "bwd_fwd_ratio": round(b_ms / f_ms, 3),
           "touched_rows": touched}
    bytes_k = {"GATHER": 2 * n * 4 + 2 * n * R * 4, "SCATTER": 2 * n * 4 + n * R * 4 + touched * R * 4,
               "GATHER_DW": 2 * n * R * 4 + 3 * n * 4}
    if j_ms is not None:
        res["jvp_ms"] = round(j_ms, 4)
        bytes_k["GATHER_JVP"] = 3 * n * 4 + 3 * n * R * 4
    for k, b in bytes_k.items():
        ms, cnt = dex.dex_profile_read(k)
        a = b / (ms / max(cnt, 1) * 1e-3) / 1e9
        res[k.lower()] = {"avg_ms": round(ms / max(cnt, 1), 4), "GBps": round(a, 1),
                          "frac_hbm": round(a / PEAK["hbm"], 4), "bytes_per_launch": b}
    del T, g, out, dT
    return res


def row_histogram(torch, dex, workloads, dev, steps):
    c = workloads.HISTOGRAM
    keys = torch.tensor(workloads.histogram_keys(c["n"], c["bins"], c["s"], c["seed"]).view("int32"),
                        device=dev)
    h = torch.zeros(c["bins"], dtype=torch.int32, device=dev)
    nb = dex.dex_accum_scatter_workspace_bytes(dex.DEX_I32, c["bins"], 1, c["n"], False)
    ws = dex.workspace(nb, dev)

    def run():
        dex.dex_accum_scatter(h, keys, ws=ws, idx_dtype=dex.DEX_U32)

    run()
    torch.cuda.synchronize()
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    ms = timed(run, steps, torch.cuda.synchronize) * 1e3
    dex.dex_profile_enable(False)
    kms, kn = dex.dex_profile_read("HIST")
    b = c["n"] * 4 + c["bins"] * 4
    a = b / (kms / max(kn, 1) * 1e-3) / 1e9
    return {"workload": f"int32 histogram of 2^26 Zipf(1.1) keys mod {c['bins']}",
            "ms": round(ms, 4), "hist_kernel": {"avg_ms": round(kms / max(kn, 1), 4), "GBps": round(a, 1),
                                                 "frac_hbm": round(a / PEAK["hbm"], 4),
                                                 "bytes_per_launch": b}}


def row_batched(torch, dex, workloads, dev, steps):
    import numpy as np
    shapes = workloads.batched_shapes()
    insts = workloads.batched_inputs(shapes)
    d, plan = dex.dex_gmm_batched_plan(shapes)
    packed = [torch.tensor(a, device=dev) for a in workloads.pack_batched(insts)]
    del insts
    tplan = torch.tensor(plan, device=dev)
    B = shapes.shape[0]
    F = torch.empty(B, device=dev)
    f = torch.empty(int(d.dims[1]), device=dev)
    cache = torch.empty(int(d.dims[7]), dtype=torch.uint8, device=dev)
    ws = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev)
    ct = torch.ones(B, device=dev)
    grads = [torch.empty_like(p) for p in packed[:4]]
    ins = [tplan, *packed]
    bf = dex.dex_autotune(d, dex.DEX_WS_FWD, ins, [F], [f, cache], [], [], ws)
    dex.dex_fwd(d, ins, [F], [f, cache], ws)
    bb = dex.dex_autotune(d, dex.DEX_WS_VJP, ins, [], [f, cache], [ct], grads, ws)

    def fwd():
        dex.dex_fwd(d, ins, [F], [f, cache], ws)

    def vjp():
        dex.dex_vjp(d, ins, [f, cache], [ct], grads, 0, ws)

    fwd()
    vjp()
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    f_ms = timed(fwd, steps, torch.cuda.synchronize) * 1e3
    b_ms = timed(vjp, steps, torch.cuda.synchronize) * 1e3
    dex.dex_profile_enable(False)
    N, D, K = shapes[:, 0], shapes[:, 1], shapes[:, 2]
    tri = float(np.sum(D * (D + 1) * N * K))
    mom = float(np.sum(D * (D + 3) * N * K))
    res = {"workload": "512 GMM instances, N~U[1000,50000], D in {8,16,32}, K~U[10,100], FP32",
           "fwd_ms": round(f_ms, 4), "vjp_ms": round(b_ms, 4), "bwd_fwd_ratio": round(b_ms / f_ms, 3),
           "grad_evals_per_s": round(1e3 / (f_ms + b_ms), 2), "config": [bf, bb],
           "algorithmic_tflop": round((tri + mom) / 1e12, 4)}
    for k, fl in (("BGMM_FWD", tri), ("BGMM_VJP", mom)):
        ms, cnt = dex.dex_profile_read(k)
        a = fl / (ms / max(cnt, 1) * 1e-3) / 1e12
        res[k.lower()] = {"avg_ms": round(ms / max(cnt, 1), 4), "tflops": round(a, 2),
                          "frac_fp32": round(a / PEAK["fp32"], 4)}
    return res


def row_stencil(torch, dex, workloads, dev, steps):
    c = workloads.STENCIL
    H, W, T, every = c["H"], c["W"], c["steps"], c["every"]
    gen = torch.Generator(device=dev).manual_seed(c["seed"])
    u0 = torch.randn(H, W, device=dev, generator=gen)
    tg = torch.randn(H, W, device=dev, generator=gen)
    out = {"workload": f"{H}x{W} f32 periodic 5-point diffusion, {T} steps, checkpoint every {every}"}
    for name, variant, fc, vc in (("recompute", dex.DEX_STENCIL_RECOMPUTE, 0, 0),
                                  ("linear", dex.DEX_STENCIL_LINEAR, 0, 0),
                                  ("recompute_vector_kernels", dex.DEX_STENCIL_RECOMPUTE, 2, 3)):
        d = dex.stencil_desc(H, W, T, every, 0.2, 0.0, variant)
        nck = (T + every - 1) // every
        L = torch.empty(1, device=dev)
        uT = torch.empty_like(u0)
        ck = torch.empty(nck * H * W, device=dev)
        wsf = dex.workspace(dex.dex_workspace_bytes(d, 0), dev)
        wsb = dex.workspace(dex.dex_workspace_bytes(d, 1), dev)
        du = torch.empty_like(u0)
        ct = torch.ones(1, device=dev)

        def fwd():
            d.config = fc
            dex.dex_fwd(d, [u0, tg], [L, uT], [ck, uT], wsf)

        def vjp():
            d.config = vc
            dex.dex_vjp(d, [u0, tg], [ck, uT], [ct], [du], 0, wsb)

        fwd()
        vjp()
        dex.dex_profile_reset()
        dex.dex_profile_enable(True)
        f_ms = timed(fwd, steps, torch.cuda.synchronize) * 1e3
        b_ms = timed(vjp, steps, torch.cuda.synchronize) * 1e3
        dex.dex_profile_enable(False)
        r = {"fwd_ms": round(f_ms, 3), "vjp_ms": round(b_ms, 3), "bwd_fwd_ratio": round(b_ms / f_ms, 3)}
        for k in ("STENCIL_FWD", "STENCIL_VJP"):
            ms, cnt = dex.dex_profile_read(k)
            per = ms / max(cnt, 1)
            a = 2 * H * W * 4 / (per * 1e-3) / 1e9
            r[k.lower()] = {"avg_ms_per_step": round(per, 5), "GBps": round(a, 1),
                            "frac_hbm": round(a / PEAK["hbm"], 4)}
        out[name] = r
        del ck, wsb
    # forward mode: primal and tangent stepped together, then dL
    d = dex.stencil_desc(H, W, T, every, 0.2, 0.0, dex.DEX_STENCIL_RECOMPUTE)
    wsj = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_JVP), dev)
    du0 = torch.randn(H, W, device=dev, generator=gen)
    tL = torch.empty(1, device=dev)

    def jvp():
        dex.dex_jvp(d, [u0, tg], [du0, tg], [tL], wsj)

    jvp()
    j_ms = timed(jvp, steps, torch.cuda.synchronize) * 1e3
    per = j_ms / max(T, 1)
    a = 4 * H * W * 4 / (per * 1e-3) / 1e9  # u, du read; u', du' written per step
    out["forward_mode"] = {"jvp_ms": round(j_ms, 3), "avg_ms_per_step": round(per, 5),
                           "GBps": round(a, 1), "frac_hbm": round(a / PEAK["hbm"], 4)}
    del wsj
    return out


def row_reduce(torch, dex, workloads, dev, steps):
    """Regular segmented reduction (2^20 rows of 128) and complete reduction
    (2^28 values), FP32 in, FP64 sums."""
    gen = torch.Generator(device=dev).manual_seed(5)
    rows, cols, n = 1 << 20, 128, 1 << 28
    v = torch.randn(rows, cols, device=dev, generator=gen)
    out = torch.empty(rows, device=dev)
    w = torch.randn(n, device=dev, generator=gen)
    o1 = torch.empty(1, device=dev)
    ws = torch.empty(dex.DEX_REDUCE_WS_BYTES, dtype=torch.uint8, device=dev)
    dex.dex_reduce_rows(out, v)
    dex.dex_reduce_all(o1, w, ws)
    torch.cuda.synchronize()
    # the kernels' own time (HIP events around each call's launches): a call
    # is shorter than its Python overhead here
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    for _ in range(steps):
        dex.dex_reduce_rows(out, v)
    for _ in range(steps):
        dex.dex_reduce_all(o1, w, ws)
    torch.cuda.synchronize()
    dex.dex_profile_enable(False)
    del v, w
    res = {"workload": f"segmented {rows}x{cols} f32 -> {rows}; complete {n} f32 -> 1"}
    for k, key, b in (("segmented", "REDUCE_ROWS", 4 * rows * cols + 4 * rows),
                      ("complete", "REDUCE_ALL", 4 * n)):
        ms, cnt = dex.dex_profile_read(key)
        per = ms / max(cnt, 1)
        a = b / (per * 1e-3) / 1e9
        res[k] = {"avg_ms": round(per, 4), "GBps": round(a, 1), "frac_hbm": round(a / PEAK["hbm"], 4),
                  "bytes_per_launch": b}
    return res


# ---------------------------------------------------------------------------
def cpu_baseline(torch, dex, workloads, g, variant, dev):
    """The FP64 oracle on two point-subsamples of the benchmark instance (all
    200 components), fitted as a + b N and evaluated at N = 1e5; plus the GPU
    gradient's error against the oracle on the larger subsample."""
    import numpy as np
    from oracle import gmm as ogmm
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    times = {}
    sub = {}
    for n in (1000, 5000):
        h = workloads.GMMInputs(g.alphas, g.means, g.qd, g.l, g.x[:n].copy())
        t0 = time.perf_counter()
        F, f = ogmm.objective(*h.params(), h.x)
        go = ogmm.vjp(*h.params(), h.x, f)
        times[n] = time.perf_counter() - t0
        sub[n] = (h, F, go)
    b = (times[5000] - times[1000]) / 4000
    a = times[1000] - b * 1000
    t_full = a + b * g.N
    h, Fo, go = sub[5000]
    S = gmm_setup(torch, dex, h, variant, dev)
    S["fwd"]()
    S["vjp"]()
    torch.cuda.synchronize()
    errs = {}
    for name, x, o in zip(("alphas", "means", "qd", "l"), S["grads"], go):
        xx = x.cpu().numpy().astype(np.float64).ravel()
        errs[name] = float(np.linalg.norm(xx - o.ravel()) / np.linalg.norm(o))
    errs["F"] = abs(S["F"].item() - Fo) / abs(Fo)
    return {"value": round(1.0 / t_full, 6), "unit": "grad evals/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle on the first 1000 and 5000 of the 100000 points (all 200 "
                      f"components, D=64), {times[1000]:.2f}s and {times[5000]:.2f}s, fitted a+bN "
                      f"and evaluated at N=100000 ({t_full:.1f}s per grad eval)"}, errs


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", choices=["bf16", "bf16x3", "fp32"], default="bf16")
    ap.add_argument("--no-rows", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--configs", default=None,
                    help="forward,reverse tile configuration (1-based); skips the autotuner")
    ap.add_argument("--rows-only", default=None, help="comma list of rows to run (scatter,hist,batched,stencil)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path has no "
              f"multi-GPU component in this build", file=sys.stderr)
        return 2
    import torch

    import workloads
    from paper_2104_05372_amd import dex
    dev = torch.device("cuda:0")
    dex.dex_init()
    log("headline: GMM gradient N=100000 D=64 K=200", args.variant)
    H = run_headline(torch, dex, workloads, args, dev)
    if args.calibration_copy:
        # a device copy of known size (256 MiB read + 256 MiB written): the
        # reference for scaling the HBM byte counters of a profiled run
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    line = {
        "metric": METRIC, "value": round(H["value"], 3), "unit": "grad evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(H["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "bf16x3": "bf16x3", "fp32": "f32"}[args.variant], "data": "synthetic",
        "config": {"workload": "gmm_grad_N100000_D64_K200", "N": 100000, "D": 64, "K": 200,
                   "products": {"bf16": "BF16 MFMA, FP32 accumulate", "bf16x3": "split-BF16 MFMA",
                                "fp32": "FP32 MFMA"}[args.variant],
                   "tile_configs": {"fwd": H["cfg"][0], "vjp": H["cfg"][1]}},
        "bwd_fwd_ratio": round(H["vjp_ms"] / H["fwd_ms"], 3),
        "fwd_ms": round(H["fwd_ms"], 4), "vjp_ms": round(H["vjp_ms"], 4),
        "roofline": H["roofline"],
    }
    g = H["g"]
    if not args.no_rows:
        # forward mode of the objective along a tangent (the gradients buffer
        # serves as the tangent): reverse pass with cotangent 1 + inner product
        S = H["S"]
        d = S["d"]
        wsj = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_JVP), dev)
        dF = torch.empty(1, device=dev)
        f = torch.empty(g.N, device=dev)
        cache = torch.empty(dex.dex_workspace_bytes(d, dex.DEX_WS_RESID), dtype=torch.uint8,
                            device=dev)
        dex.dex_fwd(d, S["t"], [S["F"]], [f, cache],
                    dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev))

        def jvp():
            dex.dex_jvp(d, S["t"], S["grads"], [dF], wsj, resid=[f, cache])

        jvp()
        j_ms = timed(jvp, max(3, args.steps // 2), torch.cuda.synchronize) * 1e3
        line["forward_mode"] = {"jvp_ms": round(j_ms, 4),
                                "form": "reverse pass with cotangent 1, then <grad F, t> in FP64"}
        del wsj, cache, S
    del H["S"]
    torch.cuda.empty_cache()
    if args.variant != "fp32":
        log("fp32 form")
        try:
            line["fp32_form"] = run_fp32_form(torch, dex, g, dev, max(3, args.steps // 4))
        except Exception as e:  # report, never hide the headline
            line["fp32_form"] = {"error": repr(e)}
    if not args.no_rows:
        rows = {}
        sel = args.rows_only.split(",") if args.rows_only else ["scatter", "scatter_det", "hist", "batched",
                                                                "stencil", "reduce"]
        fns = {"scatter": row_scatter, "hist": row_histogram, "batched": row_batched, "stencil": row_stencil,
               "reduce": row_reduce,
               "scatter_det": lambda *a: row_scatter(*a, scatter_config=2)}
        for name in sel:
            log("row", name)
            try:
                rows[name] = fns[name](torch, dex, workloads, dev, 5 if name != "stencil" else 2)
            except Exception as e:
                rows[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
        line["rows"] = rows
    if not args.no_cpu_baseline:
        log("cpu baseline")
        variant = {"bf16": dex.DEX_GMM_BF16, "bf16x3": dex.DEX_GMM_BF16X3, "fp32": dex.DEX_GMM_PLAIN}[args.variant]
        try:
            cb, errs = cpu_baseline(torch, dex, workloads, g, variant, dev)
            line["cpu_baseline"] = cb
            line["rel_l2_vs_fp64_oracle"] = {k: float(f"{v:.3e}") for k, v in errs.items()}
        except Exception as e:
            line["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
