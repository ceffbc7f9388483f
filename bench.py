#!/usr/bin/env python3
"""Benchmark of the scatter-accumulate reverse-mode path on one MI355X.

A step is one GMM gradient evaluation (dex_fwd + dex_vjp: F and the cotangents
of alphas, means, qd and l) at N=100000, D=64, K=200 with 16-bit matrix-core
operands (FP16 at D = 64) and FP32 accumulation, inputs resident in HBM. The
timed steps run with nothing else enqueued between them. Prints one JSON line.

The line also carries, measured in the same run:
  roofline      the dominant kernel's algorithmic FLOP rate against the 16-bit
                dense peak, its duration taken with HIP events around each
                launch in a separate pass;
  forward_mode  the derivative of the objective along a tangent (dex_jvp);
  bf16_resident_form, fp32_form  the same gradient with BF16 Q~(x~ - mu~)
                products, and with FP32 matrix-core products;
  rows          the other workloads of the path (gather / scatter-accumulate,
                histogram, batched GMM, checkpointed stencil adjoint,
                reductions), each with its kernel time and roofline fraction;
  cpu_baseline  the FP64 oracle timed on this host: one full-size evaluation on
                all threads, and a one-thread sample; rel_l2_vs_fp64_oracle is
                the headline's error against that full-size evaluation.
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


CHECK = {"on": True}  # the rows' oracle checks (off for profiling runs)


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu_timed(fn):
    t0 = time.perf_counter()
    r = fn()
    return r, time.perf_counter() - t0


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
    # 1) the timed steps: nothing but the two calls (no events, profiling off)
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sync()
    elapsed = time.perf_counter() - t0
    # 2) forward / reverse split, with events between the calls
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e in ev:
        e[0].record()
        S["fwd"]()
        e[1].record()
        S["vjp"]()
        e[2].record()
    sync()
    fwd_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / len(ev)
    vjp_ms = sum(b.elapsed_time(c) for _, b, c in ev) / len(ev)
    # 3) the main kernels' own durations (HIP events around each launch)
    dex.dex_profile_reset()
    dex.dex_profile_enable(True)
    for _ in range(args.steps):
        step()
    sync()
    dex.dex_profile_enable(False)
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
                          "weighted moment sum_i w x x^T and sum_i w x per component)",
            "timing": "kernel durations from HIP events around each launch, in a pass of their "
                      "own after the timed steps"}
    res = dict(value=args.steps / elapsed, ms=elapsed / args.steps * 1e3, fwd_ms=fwd_ms, vjp_ms=vjp_ms,
               roofline=roof, cfg=S["cfg"], g=g, S=S)
    return res


def headline_vs_oracle(torch, dex, g, S, threads):
    """One FP64 oracle evaluation (objective + gradient) of the whole benchmark
    instance on the host, timed: the CPU baseline at full size, and the
    reference for the GPU result's error (the GPU state holds the last step)."""
    import numpy as np
    from oracle import gmm as ogmm
    torch.cuda.synchronize()
    got = [x.cpu().numpy().astype(np.float64) for x in S["grads"]]
    Fg = float(S["F"].item())
    t0 = time.perf_counter()
    Fo, fo = ogmm.objective(*g.params(), g.x)
    go = ogmm.vjp(*g.params(), g.x, fo)
    secs = time.perf_counter() - t0
    errs = {n: float(np.linalg.norm(a.ravel() - o.ravel()) / np.linalg.norm(o))
            for n, a, o in zip(("alphas", "means", "qd", "l"), got, go)}
    errs["F"] = abs(Fg - Fo) / abs(Fo)
    return secs, errs


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
def row_scatter(torch, dex, workloads, dev, steps, scatter_config=1, check=True):
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
           "scatter_form": {1: "radix sort, one owner per row, no atomics",
                            2: "block sort + run sums + atomics"}[scatter_config],
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
    if check and CHECK["on"]:
        res.update(scatter_vs_oracle(torch, idx_np, T, w, g, out, dT, dw, fwd, vjp, V))
    del T, g, out, dT
    return res


def scatter_vs_oracle(torch, idx_np, T, w, g, out, dT, dw, fwd, vjp, V):
    """The reverse pass's cotangent rows of a sample of rows (the three hottest,
    61 others drawn among the touched rows, 4 untouched) and 64 sampled dw_j and
    gathered rows, against the FP64 oracle applied to the entries they depend on;
    and the oracle's own time on the first 2^18 indices, scaled to all of them."""
    import numpy as np
    from oracle import scatter as osc
    fwd()
    vjp()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows, cnt = np.unique(idx_np, return_counts=True)
    hot = rows[np.argsort(-cnt)[:3]]
    untouched = np.setdiff1d(np.arange(2000), rows)[:4]
    sample = np.concatenate([hot, rng.choice(rows, 61, replace=False), untouched])
    order = np.argsort(idx_np, kind="stable")
    sidx = idx_np[order]
    dT_s = dT[torch.tensor(sample.astype(np.int64), device=dT.device)].cpu().numpy()
    w_np = w.cpu().numpy()
    want = []
    for v in sample:
        a, b = np.searchsorted(sidx, v), np.searchsorted(sidx, v, side="right")
        js = order[a:b]
        gs = g[torch.tensor(js.astype(np.int64), device=g.device)].cpu().numpy()
        want.append(osc.scatter_rows([v], idx_np[js], w_np[js], gs)[0])
    js = rng.integers(0, idx_np.size, 64)
    jt = torch.tensor(js.astype(np.int64), device=g.device)
    Ts = T[torch.tensor(idx_np[js].astype(np.int64), device=T.device)].cpu().numpy()
    gs = g[jt].cpu().numpy()
    loc = np.arange(64)
    err = {"dT_sampled_rows": rel_l2(dT_s, np.array(want)),
           "dw_sampled": rel_l2(dw[jt].cpu().numpy(), osc.scatter_dw(Ts, loc, gs)),
           "out_sampled": rel_l2(out[jt].cpu().numpy(), osc.gather(Ts, loc, w_np[js]))}
    m = 1 << 18
    g_m = g[:m].cpu().numpy()
    _, t = cpu_timed(lambda: osc.scatter(V, idx_np[:m], w_np[:m], g_m))
    n = idx_np.size
    return {"rel_l2_vs_fp64_oracle": {k: float(f"{v:.3e}") for k, v in err.items()},
            "cpu_oracle": {"ms_per_call": round(t * n / m * 1e3, 1), "cores": 1,
                           "sample": f"FP64 oracle scatter on the first {m} of {n} indices, "
                                     f"{t:.2f} s, times {n // m} (one thread; the sample includes "
                                     f"the table's FP64 zero fill)"}}


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
    res = {"workload": f"int32 histogram of 2^26 Zipf(1.1) keys mod {c['bins']}",
           "ms": round(ms, 4), "hist_kernel": {"avg_ms": round(kms / max(kn, 1), 4), "GBps": round(a, 1),
                                                "frac_hbm": round(a / PEAK["hbm"], 4),
                                                "bytes_per_launch": b}}
    if not CHECK["on"]:
        return res
    import numpy as np
    from oracle import scatter as osc
    h.zero_()
    run()
    got = h.cpu().numpy()
    keys_np = keys.cpu().numpy().view(np.uint32)
    want, t = cpu_timed(lambda: osc.histogram(keys_np, c["bins"]))
    res["bit_exact_vs_oracle"] = bool(np.array_equal(got, want))
    res["cpu_oracle"] = {"ms_per_call": round(t * 1e3, 1), "cores": 1,
                         "sample": "FP64/int64 oracle on all 2^26 keys (one thread)"}
    return res


def row_batched(torch, dex, workloads, dev, steps):
    import numpy as np
    shapes = workloads.batched_shapes()
    insts = workloads.batched_inputs(shapes)
    packed = [torch.tensor(a, device=dev) for a in workloads.pack_batched(insts)]
    del insts
    B = shapes.shape[0]
    N, D, K = shapes[:, 0], shapes[:, 1], shapes[:, 2]
    tri = float(np.sum(D * (D + 1) * N * K))
    mom = float(np.sum(D * (D + 3) * N * K))

    def measure(variant):
        """Autotuned forward and reverse of the whole batch in one variant: the
        timings, the kernel figures and the outputs of one more evaluation."""
        d, plan = dex.dex_gmm_batched_plan(shapes, variant)
        tplan = torch.tensor(plan, device=dev)
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
        r = {"fwd_ms": round(f_ms, 4), "vjp_ms": round(b_ms, 4), "bwd_fwd_ratio": round(b_ms / f_ms, 3),
             "grad_evals_per_s": round(1e3 / (f_ms + b_ms), 2), "config": [bf, bb]}
        for k, fl in (("BGMM_FWD", tri), ("BGMM_VJP", mom)):
            ms, cnt = dex.dex_profile_read(k)
            a = fl / (ms / max(cnt, 1) * 1e-3) / 1e12
            r[k.lower()] = {"avg_ms": round(ms / max(cnt, 1), 4), "tflops": round(a, 2),
                            "frac_fp32": round(a / PEAK["fp32"], 4)}
        out = None
        if CHECK["on"]:
            fwd()
            vjp()
            torch.cuda.synchronize()
            out = (F.cpu().numpy(), f.cpu().numpy(), [x.cpu().numpy() for x in grads])
        del cache, ws, grads, tplan
        torch.cuda.empty_cache()
        return r, out

    res, out = measure(dex.DEX_GMM_PLAIN)
    res = {"workload": "512 GMM instances, N~U[1000,50000], D in {8,16,32}, K~U[10,100], FP32",
           **res, "algorithmic_tflop": round((tri + mom) / 1e12, 4)}
    # the split-FP16 form of the same batch (instances with D > 8 take hi + lo
    # FP16 operands, scaled into range; FP32-class results)
    res_s, out_s = measure(dex.DEX_GMM_F16X3)
    for k in ("bgmm_fwd", "bgmm_vjp"):
        a = res_s[k]["tflops"]
        res_s[k]["frac_fp16_over_3"] = round(a / (PEAK["bf16"] / 3), 4)
    res_s["products"] = ("D > 8: forward on split FP16 operands (hi*hi + hi*lo + lo*hi, FP32 "
                         "accumulation, power-of-two scaled), reverse FP32 moments; D <= 8 as FP32")
    res["split_fp16"] = res_s
    if not CHECK["on"]:
        return res
    # a sample of instances against the FP64 oracle (the largest, the smallest
    # and two others), and the oracle's time on them scaled by algorithmic cost
    from oracle import gmm as ogmm
    cost = N * K * D * D
    pick = sorted({int(np.argmax(cost)), int(np.argmin(cost)), 0, B // 2})
    offs = {name: np.concatenate([[0], np.cumsum(v)]) for name, v in
            (("N", N), ("K", K), ("KD", K * D), ("KL", K * D * (D - 1) // 2))}
    errs, errs_s, t_cpu = [], [], 0.0
    sl = lambda key, i: slice(offs[key][i], offs[key][i + 1])
    for b in pick:
        gi = workloads.gmm_inputs(int(N[b]), int(D[b]), int(K[b]), workloads.BATCHED["seed"] + 1 + b,
                                  np.float32)
        (Fo, fo), t1 = cpu_timed(lambda: ogmm.objective(*gi.params(), gi.x))
        go, t2 = cpu_timed(lambda: ogmm.vjp(*gi.params(), gi.x, fo))
        t_cpu += t1 + t2
        for (Fg, fg, gg), e in ((out, errs), (out_s, errs_s)):
            blk = [gg[0][sl("K", b)], gg[1][sl("KD", b)], gg[2][sl("KD", b)], gg[3][sl("KL", b)]]
            e.append(max([abs(Fg[b] - Fo) / abs(Fo), rel_l2(fg[sl("N", b)], fo)] +
                         [rel_l2(a, o) for a, o in zip(blk, go) if o.size]))
    scale = float(cost.sum() / cost[pick].sum())
    res["rel_l2_vs_fp64_oracle"] = {"max_over_sampled_instances": float(f"{max(errs):.3e}"),
                                    "instances": pick}
    res["split_fp16"]["rel_l2_vs_fp64_oracle"] = {
        "max_over_sampled_instances": float(f"{max(errs_s):.3e}"), "instances": pick}
    res["cpu_oracle"] = {"ms_per_grad_eval": round(t_cpu * scale * 1e3, 1), "cores": blas_threads(),
                         "sample": f"FP64 oracle on instances {pick} ({t_cpu:.2f} s), scaled by "
                                   f"the batch's N K D^2 over theirs ({scale:.1f}x)"}
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
    if not CHECK["on"]:
        return out
    # the same grid and kernels for 8 steps (checkpoint every 4, so the reverse
    # pass recomputes) against the FP64 oracle loop; its time scaled to 1000 steps
    from oracle import stencil as ost
    Ts, es = 8, 4
    d = dex.stencil_desc(H, W, Ts, es, 0.2, 0.0, dex.DEX_STENCIL_RECOMPUTE)
    L = torch.empty(1, device=dev)
    uT = torch.empty_like(u0)
    ck = torch.empty((Ts // es) * H * W, device=dev)
    du = torch.empty_like(u0)
    dex.dex_fwd(d, [u0, tg], [L, uT], [ck, uT], dex.workspace(dex.dex_workspace_bytes(d, 0), dev))
    dex.dex_vjp(d, [u0, tg], [ck, uT], [torch.ones(1, device=dev)], [du], 0,
                dex.workspace(dex.dex_workspace_bytes(d, 1), dev))
    torch.cuda.synchronize()
    (Lo, uTo, duo), t = cpu_timed(lambda: ost.loss_and_grad(u0.cpu().numpy(), tg.cpu().numpy(), Ts))
    out["rel_l2_vs_fp64_oracle"] = {"L": float(f"{abs(L.item() - Lo) / abs(Lo):.3e}"),
                                    "uT": float(f"{rel_l2(uT.cpu().numpy(), uTo):.3e}"),
                                    "du0": float(f"{rel_l2(du.cpu().numpy(), duo):.3e}"),
                                    "at": f"{H}x{W}, {Ts} steps, checkpoint every {es}"}
    out["cpu_oracle"] = {"ms_per_1000_steps_fwd_and_vjp": round(t * 1000 / Ts * 1e3, 1),
                         "cores": blas_threads(),
                         "sample": f"FP64 oracle loop and its transpose, {Ts} steps on the {H}x{W} "
                                   f"grid ({t:.2f} s), times {1000 // Ts}"}
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
    res = {"workload": f"segmented {rows}x{cols} f32 -> {rows}; complete {n} f32 -> 1"}
    for k, key, b in (("segmented", "REDUCE_ROWS", 4 * rows * cols + 4 * rows),
                      ("complete", "REDUCE_ALL", 4 * n)):
        ms, cnt = dex.dex_profile_read(key)
        per = ms / max(cnt, 1)
        a = b / (per * 1e-3) / 1e9
        res[k] = {"avg_ms": round(per, 4), "GBps": round(a, 1), "frac_hbm": round(a / PEAK["hbm"], 4),
                  "bytes_per_launch": b}
    if not CHECK["on"]:
        del v, w
        return res
    # 4096 sampled rows and the complete sum of the first 2^24 values (a call of
    # its own) against the FP64 oracle (math.fsum); the oracle's time scaled up
    import numpy as np
    from oracle import reduce as ored
    rs = np.random.default_rng(1).integers(0, rows, 4096)
    vs = v[torch.tensor(rs, device=dev)].cpu().numpy()
    want_rows, t_rows = cpu_timed(lambda: ored.reduce_rows(vs))
    m = 1 << 24
    o2 = torch.empty(1, device=dev)
    dex.dex_reduce_all(o2, w[:m].contiguous(), ws)
    wm = w[:m].cpu().numpy()
    want_all, t_all = cpu_timed(lambda: ored.reduce_all(wm))
    res["rel_l2_vs_fp64_oracle"] = {"segmented_sampled_rows": float(f"{rel_l2(out[torch.tensor(rs, device=dev)].cpu().numpy(), want_rows):.3e}"),
                                    "complete_first_2^24": float(f"{abs(o2.item() - want_all) / max(abs(want_all), 1e-300):.3e}")}
    res["cpu_oracle"] = {"segmented_ms": round(t_rows * rows / 4096 * 1e3, 1),
                         "complete_ms": round(t_all * n / m * 1e3, 1), "cores": 1,
                         "sample": f"math.fsum over 4096 rows ({t_rows:.2f} s, times {rows // 4096}) "
                                   f"and over 2^24 values ({t_all:.2f} s, times {n // m})"}
    del v, w
    return res


# ---------------------------------------------------------------------------
def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_single_thread(g, n_sample=5000):
    """The FP64 oracle on one thread over the first n_sample points (all
    components); its cost is linear in N, so the full-size time is the sample
    time times N / n_sample."""
    from oracle import gmm as ogmm
    import workloads
    h = workloads.GMMInputs(g.alphas, g.means, g.qd, g.l, g.x[:n_sample].copy())
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1)
    except Exception:
        ctx = None
    t0 = time.perf_counter()
    try:
        _, f = ogmm.objective(*h.params(), h.x)
        ogmm.vjp(*h.params(), h.x, f)
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else ctx.__exit__(None, None, None)
    t = time.perf_counter() - t0
    return t, t * g.N / n_sample


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--variant", choices=["bf16", "bf16x3", "fp32"], default="bf16")
    ap.add_argument("--no-rows", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--configs", default=None,
                    help="forward,reverse tile configuration (1-based); skips the autotuner")
    ap.add_argument("--rows-only", default=None,
                    help="comma list of rows to run (scatter,scatter_atomic,hist,batched,stencil,reduce); "
                         "with --skip-headline, only these run (for profiling a row's kernels)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the rows' oracle checks and CPU timings (profiling runs)")
    ap.add_argument("--skip-headline", action="store_true",
                    help="profiling aid: run only the rows named by --rows-only and print them")
    args = ap.parse_args(argv)
    CHECK["on"] = not args.no_check
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has "
              f"no multi-GPU path", file=sys.stderr)
        return 2
    import torch

    import workloads
    from paper_2104_05372_amd import dex
    dev = torch.device("cuda:0")
    dex.dex_init()
    if args.skip_headline:
        fns = {"scatter": row_scatter, "hist": row_histogram, "batched": row_batched,
               "stencil": row_stencil, "reduce": row_reduce,
               "scatter_atomic": lambda *a: row_scatter(*a, scatter_config=2)}
        rows = {}
        for name in (args.rows_only or "").split(","):
            if name:
                log("row", name)
                rows[name] = fns[name](torch, dex, workloads, dev, 5 if name != "stencil" else 2)
                torch.cuda.empty_cache()
        print(json.dumps({"rows": rows}), flush=True)
        return 0
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
        "dtype": {"bf16": "fp16", "bf16x3": "bf16x3", "fp32": "f32"}[args.variant], "data": "synthetic",
        "config": {"workload": "gmm_grad_N100000_D64_K200", "N": 100000, "D": 64, "K": 200,
                   "products": {"bf16": "16-bit variant: forward one FP16 matrix-core product over "
                                        "second-order features (per-tile power-of-two scaling), "
                                        "reverse FP16 weighted moments, FP32 accumulation",
                                "bf16x3": "split-BF16 MFMA", "fp32": "FP32 MFMA"}[args.variant],
                   "tile_configs": {"fwd": H["cfg"][0], "vjp": H["cfg"][1]}},
        "bwd_fwd_ratio": round(H["vjp_ms"] / H["fwd_ms"], 3),
        "fwd_ms": round(H["fwd_ms"], 4), "vjp_ms": round(H["vjp_ms"], 4),
        "roofline": H["roofline"],
    }
    g = H["g"]
    if not args.no_rows:
        # forward mode of the objective along a tangent (the gradients buffer
        # serves as the tangent): the linearized loop run forward
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
        nj = max(3, args.steps // 2)
        j_ms = timed(jvp, nj, torch.cuda.synchronize) * 1e3
        dex.dex_profile_reset()
        dex.dex_profile_enable(True)
        for _ in range(nj):
            jvp()
        torch.cuda.synchronize()
        dex.dex_profile_enable(False)
        kms, kn = dex.dex_profile_read("GMM_JVP")
        tri = g.D * (g.D + 1) * g.N * g.K
        kt = tri / (kms / max(kn, 1) * 1e-3) / 1e12
        line["forward_mode"] = {
            "jvp_ms": round(j_ms, 4),
            "tangent_kernel": {"avg_ms": round(kms / max(kn, 1), 4), "tflops": round(kt, 2),
                               "frac": round(kt / PEAK["bf16"], 4)},
            "form": "linearized loop run forward: tangent coefficients (dP = dQ^T Q + Q^T dQ), one "
                    "FP16 matrix-core product over the forward's second-order features, weighted "
                    "by exp(beta - f) from the forward's residuals; no reverse pass"}
        del wsj, cache, S
        # the BF16 products the workload names (Q~ (x~ - mu~), the resident-component
        # forward, tile configuration 2) in place of the feature-product forward
        try:
            SB = gmm_setup(torch, dex, g, dex.DEX_GMM_BF16, dev, (2, H["cfg"][1]))
            for _ in range(2):
                SB["fwd"]()
                SB["vjp"]()
            ms = timed(lambda: (SB["fwd"](), SB["vjp"]()), max(3, args.steps // 2),
                       torch.cuda.synchronize) * 1e3
            line["bf16_resident_form"] = {
                "grad_evals_per_s": round(1e3 / ms, 2), "ms_per_step": round(ms, 4),
                "products": "forward BF16 Q~(x~ - mu~) (4 components resident per wave), "
                            "reverse FP16 weighted moments"}
            del SB
        except Exception as e:
            line["bf16_resident_form"] = {"error": repr(e)}
    H["S_keep"] = {"F": H["S"]["F"], "grads": H["S"]["grads"]}  # the headline's result
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
        sel = args.rows_only.split(",") if args.rows_only else ["scatter", "scatter_atomic", "hist",
                                                                "batched", "stencil", "reduce"]
        fns = {"scatter": row_scatter, "hist": row_histogram, "batched": row_batched, "stencil": row_stencil,
               "reduce": row_reduce,
               "scatter_atomic": lambda *a: row_scatter(*a, scatter_config=2)}
        for name in sel:
            log("row", name)
            try:
                rows[name] = fns[name](torch, dex, workloads, dev, 5 if name != "stencil" else 2)
            except Exception as e:
                rows[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
        line["rows"] = rows
    if not args.no_cpu_baseline:
        # one full-size FP64 oracle evaluation on all host threads (the CPU
        # baseline, and the reference for the headline's error), plus a
        # single-thread sample
        log("cpu baseline")
        try:
            secs, errs = headline_vs_oracle(torch, dex, g, H["S_keep"], blas_threads())
            t1, t1_full = cpu_single_thread(g)
            line["cpu_baseline"] = {
                "value": round(1.0 / secs, 6), "unit": "grad evals/s", "cores": blas_threads(),
                "kind": "oracle",
                "sample": f"one FP64 oracle evaluation (objective + gradient) of the whole "
                          f"N=100000, D=64, K=200 instance on {blas_threads()} host threads, "
                          f"{secs:.1f} s; host CPU {cpu_model()}, {os.cpu_count()} logical CPUs",
                "single_thread": {"value": round(1.0 / t1_full, 6), "unit": "grad evals/s",
                                  "sample": f"first 5000 points, one thread, {t1:.2f} s, times "
                                            f"N/5000 (the cost is linear in N)"}}
            line["rel_l2_vs_fp64_oracle"] = {k: float(f"{v:.3e}") for k, v in errs.items()}
            line["rel_l2_vs_fp64_oracle"]["at"] = "full size, the last timed step's result"
        except Exception as e:
            line["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
