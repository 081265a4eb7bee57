#!/usr/bin/env python3
"""Throughput of the QTT denoising-convolution pipeline on one MI355X.

One step = decompose the signal (TT-SVD, eps, rank cap), build the QTT of
the sinc Toeplitz generator, convolve in QTT format, round, reconstruct the
2^d outputs -- every stage in the HIP library, input resident in HBM.

Prints ONE JSON line (rank 0):
  value       = samples/s = 2^d * steps / wall time of the timed steps
  roofline    = the kernel class with the largest GPU time per step, its
                algorithmic work per launch over its average launch time
                (HIP events recorded on the launch stream by the library)
  cpu_baseline= the FP64 CPU oracle (same pipeline, same input) timed on the
                host cores on a bounded number of repetitions
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector / matrix
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense bfloat16 matrix
N_CU = 256

WORKLOADS = {
    # 1-D range line, 64 scatterers on a cosine background, 5% noise
    "line_d20": dict(d=20, B=2000.0, max_rank=32, seed=2),
    "line_d16": dict(d=16, B=500.0, max_rank=32, seed=2),
    # 4096 independent lines of 2^10..2^16 samples, per-line bandwidths, FP32
    "batch4096": dict(n_lines=4096, d_lo=10, d_hi=16, max_rank=32, seed=4),
    # 4096 x 4096 SAR-like image, separable sinc kernel, FP32, BF16 sketch rounding
    "image4096": dict(image=12, B=1000.0, max_rank=32, seed=3, eps=1e-3, ell=64),
    # K = 8 modes of size 10, uniform entries: TT-SVD against max-rank TT-RSVD
    "modes_k8_m10": dict(modes_K=8, M=10, max_rank=10, oversample=10, seed=8),
    # the paper's own route (Algorithm 2 with QTT-FFT in Step 3) on Example 1 at
    # K = 20: max-rank TT-SVD R_max = 10, QFFT/QiFFT truncated at R^_max = 15
    "qfft_example1_k20": dict(qfft_K=20, max_rank=10, max_rank_hat=15, eps=1e-4,
                              oversample=8, seed=1),
    # the same route on Example 3, the 2-D image at K = 10 (two-dimensional
    # transforms, one axis block each)
    "qfft_example3_k10": dict(qfft_K=10, qfft_2d=True, max_rank=10, max_rank_hat=15, eps=1e-4,
                              oversample=8, seed=1),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="line_d20", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget for the CPU oracle baseline (0 disables it)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, run one plain device copy of this many MiB "
                         "(a known-size kernel for scaling hardware byte counters)")
    ap.add_argument("--round-compare", action="store_true",
                    help="also time TT-rounding of the convolution output in QTT format "
                         "(QR and SVD sweeps of its cores by torch.linalg / rocSOLVER) "
                         "against the library's rounding (Full, then the TT-SVD sweep)")
    ap.add_argument("--breakdown", action="store_true",
                    help="also report GPU time per step of every kernel class")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2301_13339_amd as q
    from synthetic import generators as G

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    wl = WORKLOADS[args.workload]
    if "n_lines" in wl:
        return bench_batch(args, wl)
    if "image" in wl:
        return bench_image(args, wl)
    if "modes_K" in wl:
        return bench_modes(args, wl)
    if "qfft_K" in wl:
        return bench_qfft(args, wl)
    d, B, R = wl["d"], wl["B"], wl["max_rank"]
    n = 1 << d
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    es = 8 if args.dtype == "f64" else 4
    noisy, clean = G.scatterers_1d(d, seed=wl["seed"])
    x = torch.tensor(noisy, dtype=tdt, device="cuda")

    def step():
        return q.pipeline(x, B, args.eps, R)

    for _ in range(max(args.warmup, 1)):
        out, st = step()
    torch.cuda.synchronize()

    # per-class GPU time of one step (events recorded by the library)
    classes = ["level_gram", "reduce", "level_eig", "project", "eig_step", "tail", "conv",
               "full_chain", "full_final", "other"]
    per_step = {}
    for c in classes:
        with q.probe(c) as p:
            step()
            torch.cuda.synchronize()
        per_step[c] = (p.ms, p.launches)
    dom = max(classes, key=lambda c: per_step[c][0])

    # the pipeline captured once into a HIP graph (every launch of both
    # streams); each replay recomputes the whole path from the resident samples
    pg = q.PipelineGraph(x, B, args.eps, R)
    for _ in range(max(args.warmup, 1)):
        pg.run()
    st = pg.stages

    # timed region: K replays back to back, nothing else recorded but one HIP
    # event pair per step on the launch stream (the side stream joins it
    # inside every step), which gives the per-step spread
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        pg.run()
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    spread = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    value = n * args.steps / (t1 - t0)
    # the same K steps launched eagerly, for reference
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t2) * 1e3 / args.steps
    # the dominant kernel class over K more steps identical to the timed ones,
    # with the library recording a HIP event pair around each of its launches
    # on the stream it is launched on
    torch.cuda.synchronize()
    with q.probe(dom) as pd:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    avg_ms = pd.ms / max(pd.launches, 1)
    launches_per_step = pd.launches / args.steps

    fr = st["f"].ranks_host()
    zr = st["z"].ranks_host()
    roof = roofline(dom, avg_ms, launches_per_step, d, es, st, args.workload, R)

    res = {
        "metric": "samples/s for QTT decompose+conv+round+reconstruct at eps=1e-4",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "launch": "HIP graph replay of the whole pipeline",
        "eager_ms_per_step": eager_ms,
        "config": {"workload": f"{args.workload}: 1-D range line N=2^{d}, 64 scatterers, "
                               f"5% noise, sinc B={B:g}, eps={args.eps:g}, rank cap {R}",
                   "d": d, "samples": n, "eps": args.eps, "max_rank": R, "B": B},
        "roofline": roof,
        "step_ms_p10_p50_p90": [spread[int(0.1 * (len(spread) - 1))],
                                spread[len(spread) // 2], spread[int(0.9 * (len(spread) - 1))]],
        # whole step against HBM: the method must read the 2^d samples once and
        # write the 2^d outputs once
        "e2e_hbm": {"algorithmic_bytes": 2 * n * es,
                    "achieved_GBs": 2 * n * es / (ms_per_step * 1e-3) / 1e9,
                    "frac": 2 * n * es / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if args.breakdown:
        res["kernels_ms_per_step"] = {c: round(v[0], 4) for c, v in per_step.items()}
        res["kernel_launches_per_step"] = {c: v[1] for c, v in per_step.items()}
        res["ranks"] = {"F": fr, "Z": zr}
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = nb
    if args.round_compare:
        res["round_in_qtt_format"] = round_compare(q, st["y"], args.eps)
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(noisy, B, args.eps, R, n, args.cpu_seconds)
    print(json.dumps(res), flush=True)


def round_compare(q, y, eps):
    """TT-rounding of the convolution output y (ranks 2 rho r) done in QTT
    format -- right-to-left LQ of every core, then left-to-right truncated
    SVDs with tau = eps ||y|| / sqrt(d-1) -- with the vendor's dense QR and SVD
    (torch.linalg on rocSOLVER), timed against the library's rounding of the
    same tensor (Full of y, then the TT-SVD sweep).  A measurement of the
    alternative, not part of the product path."""
    import torch
    cores = [torch.tensor(c, device="cuda") for c in y.core_list()]
    D = len(cores)

    def qtt_format_round(G):
        G = [g.clone() for g in G]
        for k in range(D - 1, 0, -1):
            r0, _, r1 = G[k].shape
            Q, Rm = torch.linalg.qr(G[k].reshape(r0, 2 * r1).T)
            G[k] = Q.T.reshape(Q.shape[1], 2, r1)
            G[k - 1] = torch.einsum("aib,bc->aic", G[k - 1], Rm.T)
        tau = eps * torch.linalg.norm(G[0]) / math.sqrt(D - 1)
        for k in range(D - 1):
            r0, _, r1 = G[k].shape
            U, sv, Vh = torch.linalg.svd(G[k].reshape(2 * r0, r1), full_matrices=False)
            tail = torch.flip(torch.cumsum(torch.flip(sv * sv, [0]), 0), [0])
            ok = torch.nonzero(tail <= tau * tau)
            r = max(int(ok[0]) if ok.numel() else sv.numel(), 1)
            G[k] = U[:, :r].reshape(r0, 2, r)
            G[k + 1] = torch.einsum("ab,bjc->ajc", sv[:r, None] * Vh[:r], G[k + 1])
        return G

    def med(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return sorted(ts)[len(ts) // 2], r

    med(lambda: q.round(y, eps, 0), 2)
    t_lib, z = med(lambda: q.round(y, eps, 0), 5)
    med(lambda: qtt_format_round(cores), 1)
    t_qf, Z = med(lambda: qtt_format_round(cores), 3)
    yr = y.ranks_host()
    qr_flops = sum(2 * (2 * yr[k + 1]) * yr[k] ** 2 - 2 * yr[k] ** 3 / 3 for k in range(1, D))
    return {"y_ranks": yr, "library_ms": t_lib, "qtt_format_ms": t_qf,
            "ranks_equal": z.ranks_host() == [1] + [g.shape[2] for g in Z],
            "qr_sweep_flops": qr_flops,
            "qr_sweep_ms_at_fp64_peak": qr_flops / (FP64_PEAK_TFLOPS * 1e12) * 1e3}


K_LEVEL = 6          # steps taken from one 64 x 64 data Gram
TAIL_ELEMS = 8192    # remainders up to this size finish in one workgroup
MAX_RANK = 64        # library rank capacity when uncapped


def eig_step_sizes(D, R, ranks):
    """Gram orders E = 2 r_{k-1} of the eig_step launches of one decomposition.

    Mirrors the library's schedule: for N = 2^D > 8192 samples, steps
    1..6 come from one 64 x 64 Gram, steps 7.. run one eig_step each until
    the remainder (2^(D-k) x 2 cap_{k-1}) fits 8192 entries, then the tail.
    """
    Reff = MAX_RANK if R == 0 else R
    cap = [1] + [min(1 << k, 1 << (D - k), Reff) for k in range(1, D)] + [1]
    if (1 << D) <= TAIL_ELEMS:
        return []
    k = K_LEVEL + 1
    while k < D and not ((1 << (D - k)) * 2 * cap[k - 1] <= TAIL_ELEMS):
        k += 1
    return [2 * ranks[j - 1] for j in range(K_LEVEL + 1, k)]


def source_digest(source=None):
    """Digest of the kernel sources a counter summary was taken on: the .hip
    file that defines the kernel (all of them when ``source`` is None) and
    every shared header."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2301_13339_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith(".hip") and source is not None and fn != source:
            continue
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(cls, workload):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current sources of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    ent = tab.get(f"{workload}:{cls}")
    if not ent or ent.get("source_digest") != source_digest(ent.get("source")):
        return None
    return ent.get("bytes_per_launch")


def roofline(cls, avg_ms, launches_per_step, d, es, st, workload, R):
    """Algorithmic work per launch of the dominant class over its average duration."""
    sec = avg_ms * 1e-3
    peak_alu = FP64_PEAK_TFLOPS if es == 8 else FP32_PEAK_TFLOPS
    traffic = measured_traffic(cls, workload)
    common = {"kernel": cls, "traffic": traffic, "avg_launch_us": avg_ms * 1e3,
              "launches_per_step": launches_per_step}
    if cls == "eig_step":
        # one launch = one truncated eigendecomposition (with vectors) of an
        # E x E Gram in ONE workgroup; work = 9 E^3 flops (symmetric QR with
        # vectors, the textbook count), averaged over the step's launches
        Es = (eig_step_sizes(d, R, st["f"].ranks_host())
              + eig_step_sizes(d + 1, 0, st["w"][0].ranks_host())
              + eig_step_sizes(d, 0, st["z"].ranks_host()))
        flops = sum(9.0 * E ** 3 for E in Es) / max(len(Es), 1)
        ach = flops / sec / 1e12
        return {"bound": "alu", "achieved": ach, "peak": peak_alu, "unit": "TFLOP/s",
                "frac": ach / peak_alu, **common,
                "work_per_launch": f"9*E^3 flops averaged over E={Es} ({flops:.4g})"}
    if cls in ("level_eig", "tail"):
        E = 64
        flops = 9.0 * E ** 3
        ach = flops / sec / 1e12
        return {"bound": "alu", "achieved": ach, "peak": peak_alu, "unit": "TFLOP/s",
                "frac": ach / peak_alu, **common,
                "work_per_launch": f"9*E^3 flops per eigensolve, E=64 ({flops:.4g})"}
    n = 1 << d
    if cls == "full_final":
        byts = n * es
        what = f"2^d outputs written ({byts} B)"
    elif cls in ("level_gram", "project"):
        byts = n * es
        what = f"2^d samples read ({byts} B)"
    else:
        return {"bound": "alu", "achieved": None, "peak": peak_alu, "unit": "TFLOP/s",
                "frac": None, **common}
    ach = byts / sec / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, **common, "work_per_launch": what}


def bench_batch(args, wl):
    """The batched form: every line through the pipeline in one graph launch,
    against a per-line loop of the single-signal GPU path."""
    import numpy as np
    import torch

    import paper_2301_13339_amd as q
    from synthetic import generators as G

    dt = torch.float32
    n, R = wl["n_lines"], wl["max_rank"]
    ds, Bs, xs, _ = G.batch_lines(n, wl["d_lo"], wl["d_hi"], wl["seed"])
    samples = sum(1 << v for v in ds)
    x = torch.tensor(np.concatenate(xs), dtype=dt, device="cuda")
    b = q.Batch(ds, Bs, dt, args.eps, R)
    out = torch.empty_like(x)
    for _ in range(max(args.warmup, 1)):
        b.run(x, out, graph=True)  # the first run tunes the chunk width and captures the graph
    torch.cuda.synchronize()
    st = b.status()
    # per-class GPU time of one run, outside the graph (the probe records events)
    classes = ["batch", "other"]
    per = {}
    for c in classes:
        with q.probe(c) as p:
            b.run(x, out, graph=False)
            torch.cuda.synchronize()
        per[c] = (p.ms, p.launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run(x, out, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = samples * args.steps / (t1 - t0)
    # baseline: per-line loop of the single-signal path over a stratified
    # sample of lines, scaled by samples
    sub = list(range(0, n, max(n // 256, 1)))
    xs_sub = [torch.tensor(xs[i], dtype=dt, device="cuda") for i in sub]
    for i, li in enumerate(sub[:8]):
        q.pipeline(xs_sub[i], Bs[li], args.eps, R)
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    for i, li in enumerate(sub):
        q.pipeline(xs_sub[i], Bs[li], args.eps, R)
    torch.cuda.synchronize()
    a1 = time.perf_counter()
    sub_samples = sum(1 << ds[i] for i in sub)
    loop_value = sub_samples / (a1 - a0)
    res = {
        "metric": "samples/s for QTT decompose+conv+round+reconstruct at eps=1e-4",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch4096: {n} independent lines of 2^{wl['d_lo']}..2^{wl['d_hi']} "
                               f"samples (8-32 scatterers, 5% noise), per-line sinc bandwidth "
                               f"U(100, 2000), eps={args.eps:g}, rank cap {R}, one graph launch",
                   "lines": n, "samples": samples},
        "per_line_loop": {"value": loop_value, "unit": "samples/s",
                          "lines_timed": len(sub), "samples_timed": sub_samples},
        "speedup_vs_loop": value / loop_value,
        "kernels_ms_per_run": {c: round(v[0], 3) for c, v in per.items()},
        "status_nonzero": int((st != 0).sum()),
        "chunk_bits": getattr(b, "chunk_bits", None),
    }
    print(json.dumps(res), flush=True)


def modes_bytes(K, M, ranks, method, R, p):
    """Algorithmic HBM bytes of one decomposition: every pass of a step reads the
    unfolding A_k (m_k x n_k doubles) once; the projection also writes R_{k+1}."""
    ell = R + p
    tot = 0
    n = M ** K
    for k in range(1, K):
        n //= M
        m = M * ranks[k - 1]
        mcap = m
        rs = method == "rsvd" and min(mcap, n) > ell
        passes = 3 if rs else 2
        tot += passes * m * n * 8 + ranks[k] * n * 8
    return tot


def bench_modes(args, wl):
    """Section 5's larger-mode experiment: a K = 8, M = 10 tensor of U[0, 1) entries
    decomposed by the max-rank TT-SVD and TT-RSVD (R = 10, p = 10).  ``value`` is the
    TT-RSVD rate; both times and the whole-decomposition HBM roofline are reported."""
    import numpy as np
    import torch

    import paper_2301_13339_amd as q

    K, M, R, p = wl["modes_K"], wl["M"], wl["max_rank"], wl["oversample"]
    n = M ** K
    g = torch.Generator(device="cuda")
    g.manual_seed(wl["seed"])
    x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    res_m = {}
    for method in ("svd", "rsvd"):
        for _ in range(max(args.warmup, 1)):
            t = q.decompose_modes(x, M, 0.0, R, method=method, oversample=p, seed=1)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        steps = max(1, min(args.steps, 10))
        e0.record()
        for _ in range(steps):
            t = q.decompose_modes(x, M, 0.0, R, method=method, oversample=p, seed=1)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res_m[method] = (ms, t.ranks_host())
    ms_r, ranks_r = res_m["rsvd"]
    ms_s, ranks_s = res_m["svd"]
    byts = modes_bytes(K, M, ranks_r, "rsvd", R, p)
    res = {
        "metric": "entries/s for the max-rank TT-RSVD of a K=8, M=10 uniform tensor",
        "value": n / (ms_r * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": max(1, min(args.steps, 10)),
        "warmup": args.warmup,
        "ms_per_step": ms_r,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: K={K} modes of size {M}, U[0,1) entries, "
                               f"max rank {R}, oversampling {p}", "K": K, "M": M,
                   "max_rank": R, "oversample": p},
        "svd_ms": ms_s,
        "rsvd_ms": ms_r,
        "ranks": {"svd": ranks_s, "rsvd": ranks_r},
        "roofline": {"bound": "hbm", "achieved": byts / (ms_r * 1e-3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": byts / (ms_r * 1e-3) / 1e9 / 8000.0,
                     "traffic": None, "kernel": "whole decomposition (TT-RSVD)",
                     "bytes_per_step": byts},
    }
    if args.cpu_seconds > 0:
        from oracle import ttm
        try:
            from threadpoolctl import threadpool_info
            threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
        except Exception:  # pragma: no cover
            threads = os.cpu_count()
        rng = np.random.default_rng(wl["seed"])
        xh = rng.random(n)
        t0 = time.perf_counter()
        ttm.tt_svd_modes(xh, [M] * K, 0.0, R, method="rsvd", oversample=p, seed=1)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / dt, "unit": "entries/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"one max-rank TT-RSVD of the full {n}-entry tensor by "
                                         f"the FP64 oracle, {dt:.1f} s"}
    print(json.dumps(res), flush=True)


def sketch_gemm_work(D, zranks, ell):
    """Algorithmic work of the sketch GEMMs of one rounding sweep: for every
    step k whose unfolding (m_k = 2 r_{k-1} rows, n_k = 2^(D-k) columns) is
    wider than the sketch (m_k > ell), Y = A Omega (2 m n ell flops, bfloat16
    operands) and B = Q^T A with B B^T (2 ell m n + 2 ell^2 n flops, FP32);
    each pass reads the unfolding once (4 m n bytes in FP32)."""
    fl_y = fl_b = byts = 0
    for k in range(1, D):
        m, n = 2 * zranks[k - 1], 1 << (D - k)
        if m > ell:
            fl_y += 2 * m * n * ell
            fl_b += 2 * ell * m * n + 2 * ell * ell * n
            byts += 2 * 4 * m * n
    return fl_y, fl_b, byts


def bench_image(args, wl):
    """The precision form on a 4096 x 4096 image: FP32 data, bfloat16-operand
    sketch rounding (matrix cores, FP32 accumulation), FP64 QR and
    eigensolvers; the error against the FP64 exact pipeline on the GPU is
    reported with it, and the exact FP32 pipeline is timed beside it."""
    import numpy as np
    import torch

    import paper_2301_13339_amd as q
    from synthetic import generators as G

    dd, B, R, eps, ell = wl["image"], wl["B"], wl["max_rank"], wl["eps"], wl["ell"]
    noisy, clean = G.sar_image_2d(dd, dd, seed=wl["seed"])
    n = noisy.size
    x = torch.tensor(noisy, dtype=torch.float32, device="cuda")

    def step():
        return q.pipeline(x, (B, B), eps, R, shape2d=noisy.shape, round_method="sketch_bf16",
                          sketch_ell=ell, sketch_seed=1)

    def exact32():
        return q.pipeline(x, (B, B), eps, R, shape2d=noisy.shape)

    for _ in range(max(args.warmup, 1)):
        out, st = step()
        exact32()
    torch.cuda.synchronize()

    def timed(fn, steps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for e0, e1 in evs:
            e0.record()
            res = fn()
            e1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) / steps, sorted(e0.elapsed_time(e1) for e0, e1 in evs), res

    wall, spread, (out, st) = timed(step, args.steps)
    wall32, spread32, _ = timed(exact32, max(3, min(args.steps, 10)))
    # GPU time per step of every kernel class (one probed step each)
    classes = ["level_gram", "reduce", "level_eig", "project", "eig_step", "tail", "conv",
               "full_chain", "full_final", "sketch", "sketch_gemm", "other"]
    per = {}
    for c in classes:
        with q.probe(c) as p:
            step()
            torch.cuda.synchronize()
        per[c] = (p.ms, p.launches)
    dom = max(classes, key=lambda c: per[c][0])
    zr = st["z"].ranks_host()
    D = 2 * dd
    fl_y, fl_b, gb = sketch_gemm_work(D, zr, ell)
    g_ms = per["sketch_gemm"][0]
    sk = {"launches_per_step": per["sketch_gemm"][1], "ms_per_step": g_ms,
          "flops_per_step": {"Y_bf16": fl_y, "BBt_f32": fl_b}, "bytes_per_step": gb}
    if g_ms > 0:
        sk["achieved_TFLOPs"] = (fl_y + fl_b) / (g_ms * 1e-3) / 1e12
        sk["frac_of_bf16_peak"] = sk["achieved_TFLOPs"] / BF16_PEAK_TFLOPS
        sk["achieved_GBs"] = gb / (g_ms * 1e-3) / 1e9
        sk["frac_of_hbm"] = sk["achieved_GBs"] / HBM_PEAK_GBS
    x64 = torch.tensor(noisy, dtype=torch.float64, device="cuda")
    ref, st64 = q.pipeline(x64, (B, B), eps, R, shape2d=noisy.shape)
    torch.cuda.synchronize()
    o, r = out.double().cpu().numpy(), ref.cpu().numpy()
    res = {
        "metric": "samples/s for QTT decompose+conv+round+reconstruct at eps=1e-3",
        "value": n / wall,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"image4096: {1 << dd} x {1 << dd} SAR-like image (200 point "
                               f"scatterers, 10 dB noise), separable sinc Bx=By={B:g}, eps={eps:g}, "
                               f"rank cap {R}, bfloat16-operand sketch rounding (ell={ell})",
                   "samples": n},
        "step_ms_p10_p50_p90": [spread[int(0.1 * (len(spread) - 1))], spread[len(spread) // 2],
                                spread[int(0.9 * (len(spread) - 1))]],
        "roofline": image_roofline(dom, per[dom], D, zr, st["f"].ranks_host(), ell),
        "sketch_gemm": sk,
        "e2e_hbm": {"algorithmic_bytes": 2 * n * 4,
                    "achieved_GBs": 2 * n * 4 / wall / 1e9,
                    "frac": 2 * n * 4 / wall / 1e9 / HBM_PEAK_GBS},
        "rel_err_vs_fp64_exact": float(np.linalg.norm(o - r) / np.linalg.norm(r)),
        "ranks": {"Z_sketch": zr, "Z_exact": st64["z"].ranks_host()},
        "exact_fp32": {"value": n / wall32, "ms_per_step": wall32 * 1e3,
                       "step_ms_p10_p50_p90": [spread32[int(0.1 * (len(spread32) - 1))],
                                               spread32[len(spread32) // 2],
                                               spread32[int(0.9 * (len(spread32) - 1))]]},
        "kernels_ms_per_step": {c: round(v[0], 4) for c, v in per.items()},
        "kernel_launches_per_step": {c: v[1] for c, v in per.items()},
    }
    print(json.dumps(res), flush=True)


def image_roofline(cls, ms_launches, D, zr, fr, ell):
    """Work per launch of the dominant class of the image step over its
    average launch time.  One-workgroup classes count 9 E^3 flops per
    eigensolve of order E (QR of the sketch: 4 m ell^2); streaming classes
    the bytes they must read."""
    ms, launches = ms_launches
    avg = ms / max(launches, 1) * 1e-3
    common = {"kernel": cls, "traffic": None, "avg_launch_us": avg * 1e6,
              "launches_per_step": launches}
    if cls in ("sketch", "eig_step", "tail", "level_eig"):
        if cls == "sketch":
            works = []
            for k in range(1, D):
                m = 2 * zr[k - 1]
                if m > ell:
                    works.append(4.0 * m * ell * ell)
                works.append(9.0 * min(m, ell) ** 3)
        else:
            works = [9.0 * (2 * r) ** 3 for r in fr[5:D - 1]] or [9.0 * 64 ** 3]
        w = sum(works) / len(works)
        ach = w / avg / 1e12
        return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_PEAK_TFLOPS, **common,
                "work_per_launch": f"{w:.4g} flops (9 E^3 per eigensolve, 4 m ell^2 per QR)"}
    return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
            **common}


def qfft_work(D, R):
    """Floating-point work of one QTT-FFT (complex FP64, 8 real flops per
    complex multiply-add): at stage s (m = D + 1 - s) the Householder QR of
    each doubled core 1..m-1 (2 k x 2 r, about 8 (2k)(2r)^2 complex flops) and
    one Jacobi SVD of each core m..2 (k x 2r; about 8 sweeps of (2r)^2 / 2
    pair rotations of 2k + 2r entries, 8 real flops each).  A model of the
    work the method needs, not a count of executed instructions."""
    fl = 0.0
    r = min(R, 16)
    for s in range(1, D + 1):
        m = D + 1 - s
        if m < 2:
            continue
        k = 1
        for p in range(1, m):
            rr = min(r, 2 ** p, 2 ** (D - p))
            M, N = 2 * k, 2 * rr
            fl += 8.0 * M * N * N
            k = min(M, N)
        for p in range(m, 1, -1):
            rr = min(r, 2 ** p, 2 ** (D - p))
            M, N = min(2 * r, 2 ** (p - 1)), 2 * rr
            fl += 8 * (N * N / 2) * (M + N) * 8.0
    return fl


def bench_qfft(args, wl):
    """Algorithm 2 with Step 3 by QTT-FFT (the paper's route) on Example 1 at
    K = 20: decompose (max-rank TT-SVD), kernel QTT, QFFT of both padded
    tensors, randomised rounding of their product, QiFFT, Full."""
    import numpy as np
    import torch

    import paper_2301_13339_amd as q
    from synthetic import generators as G

    K, R, Rh, eps = wl["qfft_K"], wl["max_rank"], wl["max_rank_hat"], wl["eps"]
    two_d = wl.get("qfft_2d", False)
    if two_d:
        noisy, clean, _, _ = G.paper_example3(K, 0)
        m = noisy.shape[0]
        xn = np.zeros((1 << K, 1 << K))
        cn = np.zeros((1 << K, 1 << K))
        xn[:m, :m] = noisy
        cn[:m, :m] = clean
        B = (1 << K) / 2.0
        n = 1 << (2 * K)
    else:
        noisy, clean, _, _ = G.paper_example1(K, 0)
        xn = np.zeros(1 << K)
        xn[: noisy.size] = noisy
        cn = np.zeros(1 << K)
        cn[: clean.size] = clean
        B = (1 << K) / 4.0
        n = 1 << K
    x = torch.tensor(xn.ravel(), device="cuda")

    def step():
        if two_d:
            return q.pipeline_fft(x, (B, B), eps, R, Rh, oversample=wl["oversample"],
                                  seed=wl["seed"], shape2d=xn.shape)
        return q.pipeline_fft(x, B, eps, R, Rh, oversample=wl["oversample"], seed=wl["seed"])

    for _ in range(max(args.warmup, 1)):
        out, st = step()
    torch.cuda.synchronize()
    per = {}
    for c in ("qfft", "qfft_hadamard", "level_gram", "reduce", "level_eig", "project",
              "eig_step", "tail", "full_chain", "full_final", "other"):
        with q.probe(c) as p:
            step()
            torch.cuda.synchronize()
        per[c] = (p.ms, p.launches)
    steps = max(1, min(args.steps, 10))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        out, st = step()
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    spread = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    from oracle import conv as OC, pipeline as P
    if two_d:
        wg = OC.toeplitz_generator(K, B)
        e2 = P.relative_error(out.cpu().numpy(), OC.toeplitz_apply_2d(cn, wg, wg))
    else:
        e2 = P.relative_error(out.cpu().numpy(), P.clean_reference_1d(cn, B))
    D = (2 * K + 2) if two_d else K + 1
    fl = qfft_work(D, Rh)
    ms_q, nq = per["qfft"]
    res = {
        "metric": "samples/s for QTT decompose+conv+reconstruct, conv by QTT-FFT (Algorithm 2)",
        "value": n * steps / (t1 - t0),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: the paper's Example 3 (2-D, noise std 0.1, "
                                f"(2^{K - 1} - 1)^2 samples padded to 2^{K} x 2^{K}), kernel "
                                f"resolution 2 dx per axis" if two_d else
                                f"{args.workload}: the paper's Example 1 (Gaussian-windowed "
                                f"sines, noise std 0.02, N = 2^{K - 1} - 1 samples padded to "
                                f"2^{K}), kernel resolution 4 dx")
                               + f", R_max = {R}, R^_max = {Rh}, complex FP64 transforms",
                   "K": K, "samples": n},
        "step_ms_p10_p50_p90": [spread[int(0.1 * (len(spread) - 1))], spread[len(spread) // 2],
                                spread[int(0.9 * (len(spread) - 1))]],
        "kernels_ms_per_step": {c: round(v[0], 3) for c, v in per.items() if v[1]},
        # the transforms are sequential chains of small QR/SVD steps run by
        # one workgroup each (two for the forward pair): the roofline is the
        # FP64 rate, of which one workgroup can use at most 1/256
        "roofline": {"bound": "alu", "kernel": "k_qfft",
                     "achieved": 3 * fl / (ms_q * 1e-3) / 1e12 if ms_q > 0 else None,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (3 * fl / (ms_q * 1e-3) / 1e12) / FP64_PEAK_TFLOPS if ms_q > 0
                     else None,
                     "traffic": None,
                     "work": f"{fl:.3e} flops per transform (model in bench.py qfft_work), "
                             f"3 transforms per step in {nq} launches"},
        "e2_vs_clean_convolution": e2,
        "paper_context": ({"table_7_1_e2_qtt0": 0.0151, "table_7_4_seconds_k10_qtt0": 0.9209,
                           "hardware": "not stated in the paper"} if two_d else
                          {"table_7_1_e2_qtt0": 0.0028, "table_7_2_seconds_k20_qtt0": 0.653,
                           "hardware": "not stated in the paper"}),
    }
    if args.cpu_seconds > 0:
        from oracle import conv, qfft as QO, tt
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
        ts = []
        t_end = time.perf_counter() + args.cpu_seconds
        while not ts or (time.perf_counter() < t_end and len(ts) < 5):
            c0 = time.perf_counter()
            F = tt.tt_svd(xn.ravel(), eps, R)
            W = tt.tt_svd(conv.toeplitz_generator(K, B), eps / 10.0)
            if two_d:
                QO.full(QO.conv_fft_2d(F, K, W, W, 0.0, Rh, 0.0, wl["oversample"],
                                       wl["seed"])).real
            else:
                QO.full(QO.conv_fft(F, W, 0.0, Rh, 0.0, wl["oversample"], wl["seed"])).real
            ts.append(time.perf_counter() - c0)
        tmed = sorted(ts)[len(ts) // 2]
        res["cpu_baseline"] = {"value": n / tmed, "unit": "samples/s", "cores": threads,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"the oracle's route (TT-SVD, kernel TT-SVD, QFFT x2, "
                                         f"randomised Hadamard rounding, QiFFT, Full) on the "
                                         f"same input, median of {len(ts)} runs, "
                                         f"{tmed:.2f} s each"}
    print(json.dumps(res), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_step_time(noisy, B, eps, R, diag_stride):
    """Wall time of the FP64 oracle pipeline with the direct convolution sum as
    block-Toeplitz matrix products (1024-sample blocks).  The decompositions,
    the rounding and Full run whole; the convolution runs on every
    ``diag_stride``-th block diagonal and its time is scaled by the ratio of
    all block pairs to the pairs computed.  The rounding takes the exact
    product (DFT route, untimed) so that its work is the full pipeline's."""
    from oracle import conv, tt
    n = noisy.size
    d = n.bit_length() - 1
    t0 = time.perf_counter()
    F = tt.tt_svd(noisy, eps, R)
    f = tt.tt_full(F)
    W = tt.tt_svd(conv.toeplitz_generator(d, B), eps / 10.0)
    wt = tt.tt_full(W)
    t1 = time.perf_counter()
    blk = min(1024, n)
    nb = n // blk
    diags = range(-(nb - 1), nb, diag_stride)
    conv.toeplitz_apply_blocked(f, wt, blk, diags)
    t2 = time.perf_counter()
    pairs = sum(nb - abs(dl) for dl in diags)
    t_conv = (t2 - t1) * (nb * nb) / pairs
    y = conv.toeplitz_apply_fft(f, wt)
    t3 = time.perf_counter()
    tt.tt_full(tt.tt_svd(y, eps))
    t4 = time.perf_counter()
    return (t1 - t0) + t_conv + (t4 - t3)


def cpu_baseline(noisy, B, eps, R, n, budget_s):
    """The FP64 oracle pipeline on the host: all BLAS threads, and one thread."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threadpool_limits = None
        threads = os.cpu_count()
    stride_all, stride_one = 8, 64
    t_all = _oracle_step_time(noisy, B, eps, R, stride_all)
    res = {"value": n / t_all, "unit": "samples/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
           "sample": f"one FP64 oracle pipeline on the same N={n} signal (TT-SVD, kernel "
                     f"TT-SVD, direct convolution sum as 1024-sample block-Toeplitz GEMMs, "
                     f"TT-SVD rounding, Full) on {threads} BLAS threads; the convolution timed "
                     f"on every {stride_all}th block diagonal and scaled to all block pairs; "
                     f"{t_all:.2f} s per step"}
    if threadpool_limits is not None and budget_s > 0:
        with threadpool_limits(limits=1):
            t_one = _oracle_step_time(noisy, B, eps, R, stride_one)
        res["single_thread"] = {"value": n / t_one, "unit": "samples/s", "cores": 1,
                                "sample": f"the same with one BLAS thread, the convolution on "
                                          f"every {stride_one}th block diagonal; {t_one:.2f} s "
                                          f"per step"}
    return res


if __name__ == "__main__":
    main()
