#!/usr/bin/env python3
"""Throughput of the online tensor-LDA hot path on one MI355X.

A step is one batch through the hot path of the batched method: the whitened
batch X = (F_B - 1 M1^T) W and one CP gradient step on Phi, either fused in
one call (tlda_whiten_cp_step, the default) or as tlda_whiten_batch followed
by tlda_cp_step (--path split).  The moment pass and the whitening refresh that
precede the CP passes are run and timed in the same process and reported
beside the steps.  Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  --gpus > 1 is not supported: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector / FP32 matrix, TFLOP/s


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--docs", type=int, default=0, help="limit the corpus size (0 = full)")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--streamed", action="store_true",
                    help="stream every step's batch from pinned host memory (tlda_stage_batch, "
                         "copy of batch i+1 overlapping the compute of batch i)")
    ap.add_argument("--path", default="fused", choices=["fused", "split"],
                    help="fused: tlda_whiten_cp_step; split: tlda_whiten_batch + tlda_cp_step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a device buffer of this many MiB (a plain copy "
                         "kernel of known size that scales the HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(corpus, spec, batches, seconds: float) -> dict:
    """The FP64 oracle (as it stands) on a bounded sample of the same batches:
    whiten 1024-document slices and take a gradient on each."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import tlda_oracle as O
    from synth import init_phi

    rng = np.random.default_rng(0)
    D, K = spec.K, spec.K
    Q, _ = np.linalg.qr(rng.standard_normal((spec.V, D)))
    W = Q * 30.0
    m = np.bincount(corpus.indices[: corpus.indptr[min(corpus.n_docs, 65536)]],
                    minlength=spec.V).astype(np.float64)
    m /= m.sum()
    Phi = init_phi(D, K, 1)
    rp, ci, va, _ = batches[0]
    step = 1024
    docs = 0
    t0 = time.perf_counter()
    s = 0
    while True:
        e = min(s + step, rp.shape[0] - 1)
        a, b = int(rp[s]), int(rp[e])
        sub_rp = (rp[s:e + 1] - a).astype(np.int64)
        X = O.whiten(sub_rp, ci[a:b], va[a:b], spec.V, m, W)
        n = O.batch_stats(sub_rp, ci[a:b], va[a:b], spec.V)["n_kept"]
        Phi = O.cp_step(X, Phi, max(n, 1), spec.alpha0, 0.0, 1e-6)
        docs += e - s
        s = e if e < rp.shape[0] - 1 else 0
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": docs / dt, "unit": "docs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{docs} documents of batch 0 ({spec.name}) in 1024-document slices, "
                      f"{dt:.1f} s: dense FP64 whitening plus the eq. vec_deriv gradient"}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if there is none for this workload or the kernel's source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get("kernels", {}).get(kernel)
    if not entry:
        return None
    src = os.path.join(ROOT, entry["source"])
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != entry["source_sha256"]:
        return None
    return entry["bytes_per_launch"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS, generate, init_phi, iter_batches

    spec = SPECS[args.workload]
    D = K = spec.K
    t = time.time()
    corpus = generate(spec, n_docs=args.docs or None)
    batches = list(iter_batches(corpus))
    log(f"[bench] generated {spec.name}: {corpus.n_docs} docs, {corpus.nnz} nnz, "
        f"{len(batches)} batches in {time.time() - t:.1f}s")

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, eig_iters=60)
    dev = [tl.CsrBatch.from_numpy(rp, ci, va) for rp, ci, va, _ in batches]
    torch.cuda.synchronize()

    # ---- moment pass (a1) and refresh, timed on the context's stream ----
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for b in dev:
        tl.tlda_update_moments(ctx, b)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_ref = time.perf_counter()
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    refresh_ms = (time.perf_counter() - t_ref) * 1e3
    moments_ms = ev[0].elapsed_time(ev[1])
    log(f"[bench] moment pass {moments_ms:.2f} ms, refresh {refresh_ms:.1f} ms")

    # ---- CP steps (a2 + a3) ----
    Phi = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
    beta = args.beta if args.beta is not None else (0.03 if spec.name == "c1" else 1e-3)
    Xbuf = torch.empty((max(b.n_rows for b in dev), D), dtype=torch.float32, device="cuda")
    nk = torch.empty(1, dtype=torch.int32, device="cuda")

    fused = args.path == "fused"

    if args.streamed:
        host = [tl.CsrBatch.from_numpy(rp, ci, va, pin=True) for rp, ci, va, _ in batches]
        staged = {}

        def batch_for(i):
            # stage batch i+1 before computing batch i, so the copy overlaps the compute
            if i not in staged:
                staged[i] = tl.tlda_stage_batch(ctx, host[i % len(host)], i % 2)
            staged[i + 1] = tl.tlda_stage_batch(ctx, host[(i + 1) % len(host)], (i + 1) % 2)
            return staged.pop(i)
    else:
        def batch_for(i):
            return dev[i % len(dev)]

    def step(i, evs=None):
        b = batch_for(i)
        if fused:
            tl.tlda_whiten_cp_step(ctx, b, beta, Phi, None, None, nk)
            if evs is not None:
                evs[1].record(stream)
                evs[2].record(stream)
        else:
            tl.tlda_whiten_batch(ctx, b, Xbuf, nk)
            if evs is not None:
                evs[1].record(stream)
            tl.tlda_cp_step(ctx, Xbuf, b.n_rows, nk, beta, Phi)
            if evs is not None:
                evs[2].record(stream)
        return b

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    K_steps = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K_steps)]
    docs = 0
    nnz_tot = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K_steps):
        evs[i][0].record(stream)
        b = step(args.warmup + i, evs[i])
        docs += b.n_rows
        nnz_tot += b.nnz
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = evs[0][0].elapsed_time(evs[-1][2])
    wh_ms = [e[0].elapsed_time(e[1]) for e in evs]
    cp_ms = [e[1].elapsed_time(e[2]) for e in evs]
    st_ms = [e[0].elapsed_time(e[2]) for e in evs]
    value = docs / (total_ms / 1e3)
    if fused:
        log(f"[bench] {K_steps} steps: {total_ms:.3f} ms (wall {wall * 1e3:.1f} ms), "
            f"fused step {np.mean(st_ms) * 1e3:.1f} us per batch")
    else:
        log(f"[bench] {K_steps} steps: {total_ms:.3f} ms (wall {wall * 1e3:.1f} ms), "
            f"whiten {np.mean(wh_ms) * 1e3:.1f} us, cp {np.mean(cp_ms) * 1e3:.1f} us per batch")

    # roofline of the dominant call
    rows_per = docs / K_steps
    csr_bytes = (4 * (docs + K_steps) + 8 * nnz_tot) / K_steps      # row_ptr, col_idx, val
    w_bytes = 4 * (spec.V * D + D)                                    # W and W^T M1, once
    cp_flops = rows_per * (4.0 * D * K + K)
    if fused:
        st_avg = float(np.mean(st_ms)) / 1e3
        ach = cp_flops / st_avg / 1e12
        roof = {"kernel": "k_whiten_cp (fused step: k_cp_penalty + k_whiten_cp + k_fused_finalize)",
                "bound": "mfma", "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS,
                "traffic": measured_traffic("k_whiten_cp", spec.name),
                "algorithmic_flops": cp_flops, "algorithmic_bytes": csr_bytes + w_bytes,
                "hbm_frac_on_algorithmic_bytes": (csr_bytes + w_bytes) / st_avg / 1e9 / HBM_PEAK_GBS,
                "avg_launch_us": st_avg * 1e6}
        wh_avg, cp_avg = float("nan"), float("nan")
    else:
        wh_bytes = csr_bytes + 4 * D * rows_per + w_bytes
        wh_avg, cp_avg = float(np.mean(wh_ms)) / 1e3, float(np.mean(cp_ms)) / 1e3
        if wh_avg >= cp_avg:
            ach = wh_bytes / wh_avg / 1e9
            roof = {"kernel": "k_whiten", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": measured_traffic("k_whiten", spec.name),
                    "algorithmic_bytes": wh_bytes, "avg_launch_us": wh_avg * 1e6}
        else:
            ach = cp_flops / cp_avg / 1e12
            roof = {"kernel": "k_cp_reduce+k_cp_finalize", "bound": "mfma", "achieved": ach,
                    "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": ach / FP32_VALU_PEAK_TFLOPS,
                    "traffic": measured_traffic("k_cp_reduce+k_cp_finalize", spec.name),
                    "algorithmic_flops": cp_flops, "avg_launch_us": cp_avg * 1e6}
    mom_docs_s = corpus.n_docs / (moments_ms / 1e3)
    # recovered topics: error to the planted ones after the timed steps
    mu, alpha, lam = tl.tlda_unwhiten(ctx, Phi, tl.TLDA_PROJECT_SIMPLEX)
    mu_h = mu.cpu().numpy()
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(mu_h[:, :, None] - corpus.mu[:, None, :]).sum(axis=0)
    r, cidx = linear_sum_assignment(cost)
    topic_l1 = float(cost[r, cidx].mean())

    out = {
        "metric": "docs/sec (whiten+CP step) at fixed topic-recovery error; % HBM roofline",
        "value": value, "unit": "docs/s", "n_gpus": 1, "steps": K_steps,
        "warmup": args.warmup, "ms_per_step": total_ms / K_steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{spec.name}: V={spec.V}, K=D={K}, alpha0={spec.alpha0}, "
                               f"{corpus.n_docs} docs of length 1+Poisson({spec.doc_len_lambda:g}), "
                               f"batch {spec.batch}, "
                               + ("streamed from pinned host memory" if args.streamed
                                  else "resident in HBM"),
                   "streamed": bool(args.streamed),
                   "global_batch": spec.batch, "beta": beta, "path": args.path},
        "roofline": roof,
        "breakdown": {"path": args.path, "step_us": float(np.mean(st_ms)) * 1e3,
                      "whiten_us": wh_avg * 1e6, "cp_step_us": cp_avg * 1e6,
                      "moment_pass_ms": moments_ms, "moments_docs_per_s": mom_docs_s,
                      "refresh_ms": refresh_ms,
                      "topic_l1_to_planted_after_steps": topic_l1},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(corpus, spec, batches, args.cpu_seconds)
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 4 * n
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
