#!/usr/bin/env python3
"""Throughput of the online tensor-LDA hot path on one MI355X.

A step is one batch through the hot path of the batched method: the whitened
batch X = (F_B - 1 M1^T) W and one CP gradient step on Phi, either fused in
one call (tlda_whiten_cp_step, the default) or as tlda_whiten_batch followed
by tlda_cp_step (--path split).  The default workload is the streaming-scale
batch shape (V = 50 000, K = D = 100, alpha0 = 2, batches of 262 144
documents of length 1 + Poisson(15)): 16 distinct batches (4 194 304
documents) resident in HBM, stepped in FP32 (the paper's arithmetic; `value`)
and, beside it on the same whitening, in BF16 (`breakdown`).  The moment pass
and the whitening refresh that precede the CP passes are run and timed in the
same process and reported beside the steps.  The K timed steps run twice:
eagerly, one library call per step, with events attached to each main
kernel's dispatch (the kernel times of the roofline), and as one captured HIP
graph of the same K steps (tlda_graph_capture_steps), replayed 3 times untimed
and then 5 times timed; the median timed replay gives `value` for the fused
path over resident batches (eager
otherwise; --streamed stages every batch from pinned host memory inside the
timed region).  An untimed fit of both precisions from the same start
reports their topic-recovery errors after the same passes.  The
tweet-shaped workload (V = 20 000, K = D = 50, 1 000 000 documents) is then
measured the same way and summarised in `breakdown.c2` (--no-c2 skips it).

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
GRAPH_REPLAYS = 5              # timed replays of the captured K steps (median reported)
GRAPH_WARM_REPLAYS = 3         # untimed replays before them (the clocks settle over ~25 ms)
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector / FP32 matrix, TFLOP/s
BF16_MFMA_PEAK_TFLOPS = 2500.0 # MI355X dense BF16 matrix, TFLOP/s


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 64 for the step workloads: the "
                    "streaming-scale kernel settles at its steady duration after a few tens "
                    "of milliseconds of steps; 1 for --online)")
    ap.add_argument("--slice-scale", type=float, default=1.0,
                    help="c4: scale factor on every slice's size")
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c5: the document-topic encoder on the tweet-shaped corpus (trained on "
                         "--train-docs solve outputs, timed on --infer-docs fresh documents)")
    ap.add_argument("--train-docs", type=int, default=2_000_000)
    ap.add_argument("--infer-docs", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--docs", type=int, default=0,
                    help="corpus size (0: 16 batches for c3, the full corpus otherwise)")
    ap.add_argument("--full-stream", action="store_true",
                    help="the whole corpus (20 000 000 documents for c3) streamed from pinned "
                         "host memory: moment pass, refresh and --cp-passes CP passes, BF16 and "
                         "then FP32 on the same whitening (PCIe-inclusive rates)")
    ap.add_argument("--cp-passes", type=int, default=3)
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the tweet-shaped summary measured after the main workload")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--streamed", action="store_true",
                    help="stream every step's batch from pinned host memory (tlda_stage_batch, "
                         "copy of batch i+1 overlapping the compute of batch i)")
    ap.add_argument("--stage-format", default="auto", choices=["auto", "f32", "u16"],
                    help="--streamed host format: u16 = 16-bit column indices and counts "
                         "(tlda_stage_batch_u16, half the PCIe bytes); auto: u16 for the BF16 "
                         "step when V <= 65536, f32 for the FP32 step")
    ap.add_argument("--path", default="fused", choices=["fused", "split"],
                    help="fused: tlda_whiten_cp_step; split: tlda_whiten_batch + tlda_cp_step")
    ap.add_argument("--precision", default="fp32", choices=["bf16", "fp32"],
                    help="precision of the timed path (the other one is timed beside it)")
    ap.add_argument("--fit-passes", type=int, default=20,
                    help="passes of the untimed fit that compares the topic-recovery error of "
                         "the two precisions")
    ap.add_argument("--fit-beta", type=float, default=None,
                    help="step size of that fit (default 0.03 for c1, 0.01 for c2, 0.001 for c3)")
    ap.add_argument("--estimator", default="centred", choices=["centred", "classic"],
                    help="classic: the alpha0-corrected moments (FP32 classic-moment context) "
                         "on c1, c2 or c3")
    ap.add_argument("--online", action="store_true",
                    help="fully online mode on c1, c2 or c3: after a batched start on the first "
                         "batch, every step is moments + warm whitening refresh + Phi rebase + "
                         "whitening and CP step of a new batch")
    ap.add_argument("--warm-iters", type=int, default=4,
                    help="subspace iterations of each warm refresh in --online")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU budget of the classic-rung and encoder baselines")
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="timed oracle runs per thread setting (median reported)")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="forked processes that generate the corpora before the GPU is first "
                         "used (1: in this process, e.g. under a profiler that sets up the GPU "
                         "before the program starts)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a device buffer of this many MiB (a plain copy "
                         "kernel of known size that scales the HBM byte counters)")
    return ap.parse_args()


def _cpu_model() -> str:
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:                     # lscpu missing: leave the model unnamed
        return "unknown"
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return "unknown"


def _host_cores() -> int:
    """Cores this process may use: the box's share when OMP_NUM_THREADS fixes
    it, else the affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(spec, batch, W, m, reps: int) -> dict:
    """The FP64 oracle's sparse path as it stands, on one full batch of the
    same workload: `whiten_csr` (SciPy CSR times W, the 1/L scale and the
    rank-one mean correction) and `cp_gradient` (NumPy BLAS contractions),
    then the update.  `reps` timed runs single-threaded and `reps` with every
    host core of this process; the median of each."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import tlda_oracle as O
    from synth import init_phi

    rp, ci, va = batch
    D, K = W.shape[1], spec.K
    Phi = init_phi(D, K, 1)

    def once() -> float:
        t0 = time.perf_counter()
        X = O.whiten_csr(rp, ci, va, spec.V, m, W)
        n = int((O.doc_lengths(rp, va) >= 3).sum())
        G = O.cp_gradient(X, Phi, max(n, 1), spec.alpha0, 0.0)
        _ = Phi - 1e-6 * G
        return time.perf_counter() - t0

    docs = rp.size - 1
    res = {}
    for label, threads in (("single", 1), ("all", _host_cores())):
        with threadpool_limits(limits=threads):
            used = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
            secs = [once() for _ in range(reps)]
        res[label] = {"docs_per_s": docs / float(np.median(secs)), "threads": int(used),
                      "runs_s": secs}
    return {"value": res["all"]["docs_per_s"], "unit": "docs/s", "cores": res["all"]["threads"],
            "kind": "oracle",
            "sample": f"one {docs}-document batch ({spec.name}), median of {reps} runs per "
                      "thread setting: the oracle's sparse FP64 whitening (CSR times W, "
                      "rank-one mean correction) plus the eq. vec_deriv gradient and update",
            "single_thread_docs_per_s": res["single"]["docs_per_s"],
            "runs_s": {"single": res["single"]["runs_s"], "all": res["all"]["runs_s"]},
            "cpu_model": _cpu_model()}


def classic_cpu_baseline(corpus, spec, batches, seconds: float) -> dict:
    """The FP64 oracle of the classic rung on a bounded sample of batch 0:
    the implicit per-document data term and gradient on 256-document slices."""
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
    Phi = init_phi(D, K, 1) * 0.3
    rp, ci, va, _ = batches[0]
    step, docs, s = 256, 0, 0
    t0 = time.perf_counter()
    while True:
        e = min(s + step, rp.shape[0] - 1)
        a, b = int(rp[s]), int(rp[e])
        sub_rp = (rp[s:e + 1] - a).astype(np.int64)
        G = O.classic_cp_gradient(sub_rp, ci[a:b], va[a:b], spec.V, m, W, Phi, spec.alpha0, 0.0)
        Phi = Phi - 1e-6 * G
        docs += e - s
        s = e if e < rp.shape[0] - 1 else 0
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": docs / dt, "unit": "docs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{docs} documents of batch 0 ({spec.name}) in 256-document slices, "
                      f"{dt:.1f} s: the classic rung's FP64 per-document data term and gradient"}


def run_classic(args) -> None:
    """The classic alpha0-corrected rung: moment pass, refresh and CP steps of
    an FP32 classic-moment context on the same corpus and batches."""
    import numpy as np
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS, generate, init_phi, iter_batches

    spec = SPECS[args.workload]
    D = K = spec.K
    corpus = generate(spec, n_docs=args.docs or None)
    batches = list(iter_batches(corpus))
    log(f"[bench] generated {spec.name}: {corpus.n_docs} docs, {corpus.nnz} nnz")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    bf16 = args.precision == "bf16"
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, classic=True, bf16=bf16, eig_iters=60)
    dev = [tl.CsrBatch.from_numpy(rp, ci, va) for rp, ci, va, _ in batches]
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for b in dev:
        tl.tlda_update_moments(ctx, b)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_ref = time.perf_counter()
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    refresh_ms = (time.perf_counter() - t_ref) * 1e3
    moments_ms = ev[0].elapsed_time(ev[1])
    log(f"[bench] classic moment pass {moments_ms:.2f} ms, refresh {refresh_ms:.1f} ms")
    beta = args.beta if args.beta is not None else 1e-3
    nk = torch.empty(1, dtype=torch.int32, device="cuda")
    Phi = torch.from_numpy((init_phi(D, K, 1) * 0.3).astype(np.float32)).cuda()
    r = run_steps(tl, ctx, lambda i: dev[i % len(dev)], True, beta, Phi, None, nk, args.steps,
                  args.warmup, stream)
    docs_per_s = r["docs"] / (r["total_ms"] / 1e3)
    kern_us = r["kern_ms"].mean(axis=0) * 1e3
    log(f"[bench] classic: {args.steps} steps {r['total_ms']:.3f} ms, step "
        f"{r['step_ms'].mean() * 1e3:.1f} us, data-term kernel {kern_us[0]:.1f} us, "
        f"{docs_per_s:.4g} docs/s")
    # roofline of the data-term kernel: one reduction row per nonzero, a D x K
    # outer product on the matrix cores; bytes = CSR + W + Z copies, once
    per = args.steps
    kname = "k_classic_cp16" if bf16 else "k_classic_cp"
    peak = BF16_MFMA_PEAK_TFLOPS if bf16 else FP32_VALU_PEAK_TFLOPS
    flops = 2.0 * (r["nnz"] / per) * D * K
    elem = 2 if bf16 else 4
    byts = (4 * (r["docs"] + per) + 8 * r["nnz"]) / per + elem * spec.V * (D + K)
    t_k = kern_us[0] / 1e6
    mm_frac = flops / t_k / 1e12 / peak
    hbm_frac = byts / t_k / 1e9 / HBM_PEAK_GBS
    if mm_frac >= hbm_frac:
        roof = {"kernel": kname, "bound": "mfma", "achieved": flops / t_k / 1e12,
                "peak": peak, "unit": "TFLOP/s", "frac": mm_frac}
    else:
        roof = {"kernel": kname, "bound": "hbm", "achieved": byts / t_k / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_frac}
    roof.update({"traffic": measured_traffic(kname, spec.name),
                 "algorithmic_flops": flops, "algorithmic_bytes": byts,
                 "mfma_frac": mm_frac, "hbm_frac": hbm_frac, "avg_launch_us": float(kern_us[0])})
    fit_beta = args.fit_beta
    if fit_beta is None:
        fit_beta = {"c1": 0.03, "c2": 0.01}.get(spec.name, 1e-3)
    Phi = torch.from_numpy((init_phi(D, K, 1) * 0.3).astype(np.float32)).cuda()
    for _ in range(args.fit_passes):
        for b in dev:
            tl.tlda_whiten_cp_step(ctx, b, fit_beta, Phi)
    l1, _ = topic_error(tl, ctx, Phi, corpus.mu)
    out = {
        "metric": "docs/sec (whiten+CP step) at fixed topic-recovery error; % HBM roofline",
        "value": docs_per_s, "unit": "docs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["total_ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if bf16 else "f32", "data": "synthetic",
        "config": {"workload": f"{spec.name} classic rung: V={spec.V}, K=D={K}, "
                               f"alpha0={spec.alpha0}, {corpus.n_docs} docs of length "
                               f"1+Poisson({spec.doc_len_lambda:g}), batch {spec.batch}, "
                               "resident in HBM",
                   "estimator": "classic", "precision": args.precision,
                   "global_batch": spec.batch, "beta": beta},
        "roofline": roof,
        "breakdown": {"step_us": float(r["step_ms"].mean()) * 1e3,
                      "main_kernel_us": [float(x) for x in kern_us],
                      "moment_pass_ms": moments_ms,
                      "moments_docs_per_s": corpus.n_docs / (moments_ms / 1e3),
                      "refresh_ms": refresh_ms},
        "accuracy": {"passes": args.fit_passes, "beta": fit_beta,
                     "classic_topic_l1_to_planted": l1},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle of the classic rung on a bounded sample")
        out["cpu_baseline"] = classic_cpu_baseline(corpus, spec, batches, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def run_online(args) -> None:
    """Fully online mode: moments, warm-started whitening refresh, Phi rebase
    and one whitening + CP step per new batch, timed per stage."""
    import numpy as np
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS, generate, init_phi, iter_batches

    spec = SPECS[args.workload]
    D = K = spec.K
    corpus = generate(spec, n_docs=args.docs or None)
    batches = list(iter_batches(corpus))
    log(f"[bench] generated {spec.name}: {corpus.n_docs} docs, {len(batches)} batches")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    bf16 = args.precision == "bf16"
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, bf16=bf16, eig_iters=60,
                         eig_warm_iters=args.warm_iters)
    dev = [tl.CsrBatch.from_numpy(rp, ci, va) for rp, ci, va, _ in batches]
    beta = args.beta if args.beta is not None else (0.03 if spec.name == "c1" else 1e-3)
    # batched start on the first batch
    tl.tlda_update_moments(ctx, dev[0], tl.TLDA_REFRESH_W)
    Phi = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
    for _ in range(3):
        tl.tlda_whiten_cp_step(ctx, dev[0], beta, Phi)
    torch.cuda.synchronize()

    def one(i, ev=None):
        b = dev[1 + i % (len(dev) - 1)] if len(dev) > 1 else dev[0]
        if ev:
            ev[0].record(stream)
        tl.tlda_update_moments(ctx, b, tl.TLDA_REFRESH_WARM)
        if ev:
            ev[1].record(stream)
        tl.tlda_rebase_phi(ctx, Phi)
        if ev:
            ev[2].record(stream)
        tl.tlda_whiten_cp_step(ctx, b, beta, Phi)
        if ev:
            ev[3].record(stream)
        return b

    for i in range(args.warmup):
        one(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    docs = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        docs += one(args.warmup + i, evs[i]).n_rows
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = evs[0][0].elapsed_time(evs[-1][3])
    stage = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs]).mean(axis=0)
    out = {
        "metric": "docs/sec (whiten+CP step) at fixed topic-recovery error; % HBM roofline",
        "value": docs / (total_ms / 1e3), "unit": "docs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if bf16 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{spec.name} fully online: V={spec.V}, K=D={K}, "
                               f"alpha0={spec.alpha0}, batch {spec.batch}, per step moments + "
                               f"warm refresh ({args.warm_iters} iterations) + rebase + "
                               "whitening and CP step, resident in HBM",
                   "mode": "online", "global_batch": spec.batch, "beta": beta},
        "roofline": None,
        "breakdown": {"moments_and_warm_refresh_ms": float(stage[0]),
                      "rebase_ms": float(stage[1]), "whiten_cp_step_ms": float(stage[2]),
                      "wall_ms": wall * 1e3},
    }
    log(f"[bench] online: {out['breakdown']}")
    print(json.dumps(out), flush=True)


def fp32_fused_kernel(D: int, K: int) -> str:
    """The FP32 fused step's kernel for this shape (D and K are padded to 16,
    32, 64, 112 or 128): the hybrid kernel when both pad to 64 or both to
    112, the wide one when either passes 64, else the small-shape kernel."""
    def bucket(n):
        return next(q for q in (16, 32, 64, 112, 128) if n <= q)
    if bucket(D) == bucket(K) and bucket(D) in (64, 112):
        return "k_whiten_cp_hyb"
    return "k_whiten_cp_wide" if D > 64 or K > 64 else "k_whiten_cp"


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


def run_steps(tl, ctx, batch_for, fused, beta, Phi, Xbuf, nk, steps, warmup, stream):
    """Untimed warm-up, then `steps` timed steps.  Events: per step around the
    whole step, and (through the library's timing hook) around its main
    kernel(s).  Returns per-step and per-kernel times in ms."""
    import numpy as np
    import torch

    def step(i):
        b = batch_for(i)
        if fused:
            tl.tlda_whiten_cp_step(ctx, b, beta, Phi, None, None, nk)
        else:
            tl.tlda_whiten_batch(ctx, b, Xbuf, nk)
            tl.tlda_cp_step(ctx, Xbuf, b.n_rows, nk, beta, Phi)
        return b

    for i in range(warmup):
        step(i)
    per = 1 if fused else 2
    ks = [torch.cuda.Event(enable_timing=True) for _ in range(per * steps)]
    ke = [torch.cuda.Event(enable_timing=True) for _ in range(per * steps)]
    for e in ks + ke:
        e.record(stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    tl.tlda_set_timing_events(ctx, ks, ke)
    docs = nnz = 0
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        b = step(warmup + i)
        evs[i][1].record(stream)
        docs += b.n_rows
        nnz += b.nnz
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tl.tlda_set_timing_events(ctx, [], [])
    total_ms = evs[0][0].elapsed_time(evs[-1][1])
    step_ms = np.array([a.elapsed_time(b) for a, b in evs])
    kern_ms = np.array([a.elapsed_time(b) for a, b in zip(ks, ke)]).reshape(steps, per)
    return {"docs": docs, "nnz": nnz, "total_ms": total_ms, "wall_ms": wall * 1e3,
            "step_ms": step_ms, "kern_ms": kern_ms}


def topic_error(tl, ctx, Phi, mu_true):
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    mu, alpha, lam = tl.tlda_unwhiten(ctx, Phi, tl.TLDA_PROJECT_SIMPLEX)
    mu = mu.cpu().numpy()
    cost = np.abs(mu[:, :, None] - mu_true[:, None, :]).sum(axis=0)
    r, c = linear_sum_assignment(cost)
    return float(cost[r, c].mean()), mu


def encoder_cpu_baseline(Xh, A, seconds: float) -> dict:
    """The oracle's projected-gradient solve (as it stands) on a bounded sample."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import tlda_oracle as O
    t0 = time.perf_counter()
    docs = 0
    while time.perf_counter() - t0 < seconds and docs < Xh.shape[0]:
        O.infer_doc_topics(Xh[docs:docs + 64], A, SOLVE_ITERS, 1e-6)
        docs += 64
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": docs / dt, "unit": "docs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{docs} whitened fresh documents, projected-gradient simplex solve "
                      f"({SOLVE_ITERS} steps max, L1-change tol 1e-6), {dt:.1f} s"}


SOLVE_ITERS = 2000        # step budget of a solve
CONVERGED_ITERS = 5000    # the converged reference (gap tolerance 0)
REFINE_STEPS = 8          # projected-gradient steps applied to every encoder output


def run_encoder(args) -> None:
    """Document-topic encoder on the tweet-shaped corpus: solve outputs of
    --train-docs documents train the encoder on the GPU; --infer-docs fresh
    documents are then assigned topic proportions by the plain solve and by
    encoder + judge, and compared."""
    import numpy as np
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS, generate, iter_batches

    spec = SPECS["c2"]
    D = K = spec.K
    n_train, n_infer = args.train_docs, args.infer_docs
    t = time.time()
    corpus = generate(spec, n_docs=n_train + n_infer)
    batches = list(iter_batches(corpus))
    log(f"[bench] generated {corpus.n_docs} documents ({n_train} training, {n_infer} fresh) "
        f"in {time.time() - t:.1f}s")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, eig_iters=60)
    n_train_batches = -(-n_train // spec.batch)
    for i, (rp, ci, va, _) in enumerate(batches[:n_train_batches]):
        tl.tlda_update_moments(ctx, tl.CsrBatch.from_numpy(rp, ci, va))
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    X = torch.empty((corpus.n_docs, D), dtype=torch.float32, device="cuda")
    for rp, ci, va, first in batches:
        n = rp.shape[0] - 1
        tl.tlda_whiten_batch(ctx, tl.CsrBatch.from_numpy(rp, ci, va), X[first:first + n])
    mu = torch.from_numpy(np.ascontiguousarray(corpus.mu)).cuda()
    torch.cuda.synchronize()
    Xtr, Xin = X[:n_train], X[n_train:].contiguous()
    # targets: the solve of the training documents, run to a duality gap of 1e-7
    t = time.perf_counter()
    Ttr, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xtr.contiguous(), n_train, mu, 1e-7, SOLVE_ITERS)
    torch.cuda.synchronize()
    log(f"[bench] training targets in {time.perf_counter() - t:.2f}s")
    # training on the GPU with the library's kernels
    H, Bt = 256, 4096
    mlp = tl.tlda_mlp_create(D, H, K, Bt)
    rng = np.random.default_rng(1234)
    init = []
    for shp in ((D, H), (H,), (H, H), (H,), (H, K), (K,)):
        lim = np.sqrt(6.0 / sum(shp)) if len(shp) == 2 else 0.0
        init.append(rng.uniform(-lim, lim, size=shp).ravel() if lim else np.zeros(shp))
    tl.tlda_mlp_set_params(mlp, np.concatenate(init).astype(np.float32))
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    steps_per_epoch = n_train // Bt
    total = steps_per_epoch * args.epochs
    g = torch.Generator(device="cpu").manual_seed(7)
    t = time.perf_counter()
    step = 0
    for ep in range(args.epochs):
        perm = torch.randperm(n_train, generator=g).cuda()
        Xs, Ts = Xtr[perm].contiguous(), Ttr[perm].contiguous()
        for b in range(steps_per_epoch):
            lr = 2e-3 * 0.5 * (1.0 + np.cos(np.pi * step / total))
            tl.tlda_mlp_train_step(mlp, Xs[b * Bt:(b + 1) * Bt], Ts[b * Bt:(b + 1) * Bt],
                                   max(lr, 1e-5), loss)
            step += 1
        torch.cuda.synchronize()
        log(f"[bench] epoch {ep + 1}: loss {float(loss.item()):.4f}")
    train_s = time.perf_counter() - t
    # equal error: each method stops at the largest duality gap for which its
    # output lands within 0.04 mean L1 of a converged solve (held-out documents)
    nv = min(32768, n_train // 8)
    Xv = Xtr[-nv:].contiguous()
    conv_v, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xv, nv, mu, 0.0, CONVERGED_ITERS)

    def calibrate(enc, min_steps):
        for cand in np.geomspace(3e-2, 1e-7, 34):       # factor ~1.47 apart
            cand = float(cand)
            th, _ = tl.tlda_infer_doc_topics_mlp(ctx, enc, Xv, nv, mu, cand, SOLVE_ITERS,
                                                 min_steps=min_steps)
            if float((th - conv_v).abs().sum(dim=1).mean()) <= 0.04:
                return cand
        return 1e-7
    tol_plain = calibrate(None, 0)
    tol_enc = calibrate(mlp, REFINE_STEPS)
    log(f"[bench] duality-gap tolerance: plain solve {tol_plain:g}, encoder {tol_enc:g}")
    # timed inference on the fresh documents: plain solve, then encoder + judge
    ref = torch.empty((n_infer, K), dtype=torch.float32, device="cuda")
    out = torch.empty_like(ref)
    ns_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
    ns = torch.zeros(1, dtype=torch.int32, device="cuda")
    w = min(65536, n_infer)
    tl.tlda_infer_doc_topics_mlp(ctx, None, Xin[:w], w, mu, tol_plain, SOLVE_ITERS, ref[:w], ns_ref)
    tl.tlda_infer_doc_topics_mlp(ctx, mlp, Xin[:w], w, mu, tol_enc, SOLVE_ITERS, out[:w], ns,
                                 min_steps=REFINE_STEPS)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    tl.tlda_infer_doc_topics_mlp(ctx, None, Xin, n_infer, mu, tol_plain, SOLVE_ITERS, ref, ns_ref)
    ev[1].record(stream)
    tl.tlda_infer_doc_topics_mlp(ctx, mlp, Xin, n_infer, mu, tol_enc, SOLVE_ITERS, out, ns,
                                 min_steps=REFINE_STEPS)
    ev[2].record(stream)
    nr = min(1_000_000, n_infer)
    raw = tl.tlda_mlp_forward(mlp, Xin[:nr])
    ev[3].record(stream)
    torch.cuda.synchronize()
    solve_ms, judged_ms, raw_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), \
        ev[2].elapsed_time(ev[3])
    # errors against a converged solve of the first fresh documents
    conv, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xin[:w], w, mu, 0.0, CONVERGED_ITERS)
    l1 = (out[:w] - conv).abs().sum(dim=1)
    l1_plain = float((ref[:w] - conv).abs().sum(dim=1).mean())
    l1_raw = float((raw[:w] - conv).abs().sum(dim=1).mean())
    value = n_infer / (judged_ms / 1e3)
    log(f"[bench] plain solve {solve_ms:.1f} ms (mean L1 {l1_plain:.4f}), encoder + judge "
        f"{judged_ms:.1f} ms ({int(ns.item())} rows stepped past {REFINE_STEPS}, mean L1 "
        f"{float(l1.mean()):.4f}), raw encoder L1 {l1_raw:.4f}")
    res = {
        "metric": "docs/sec document-topic inference (encoder + judge) at mean L1 <= 0.04 "
                  "to the converged simplex solve",
        "value": value, "unit": "docs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": judged_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"encoder d={D}->{H}->{H}->{K} on the tweet-shaped corpus "
                               f"(V={spec.V}): {n_train} training pairs, {n_infer} fresh documents",
                   "train_docs": n_train, "infer_docs": n_infer, "epochs": args.epochs,
                   "batch": Bt},
        "breakdown": {"solve_docs_per_s": n_infer / (solve_ms / 1e3),
                      "speedup_over_solve": solve_ms / judged_ms,
                      "raw_encoder_docs_per_s": nr / (raw_ms / 1e3),
                      "mean_l1_to_converged": float(l1.mean()),
                      "p99_l1_to_converged": float(torch.quantile(l1, 0.99)),
                      "plain_solve_mean_l1_to_converged": l1_plain,
                      "raw_encoder_mean_l1": l1_raw,
                      "refine_steps": REFINE_STEPS,
                      "stepped_past_refine_fraction": int(ns.item()) / n_infer,
                      "gap_tol_encoder": tol_enc, "gap_tol_plain": tol_plain,
                      "train_seconds": train_s,
                      "final_train_loss": float(loss.item())},
    }
    if not args.no_cpu_baseline:
        from oracle import tlda_oracle as O
        W, _, m = tl.tlda_get_whitening(ctx)
        A = O.inference_matrix(np.ascontiguousarray(corpus.mu), m, W)
        res["cpu_baseline"] = encoder_cpu_baseline(Xin[:4096].cpu().numpy().astype(np.float64), A,
                                                   args.cpu_seconds)
    print(json.dumps(res), flush=True)


def _fork_map(fn, items, workers: int) -> list:
    """map over forked workers (before the process first uses the GPU), or
    in this process when workers <= 1; the workers leave on their own."""
    if workers <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(min(workers, len(items)))
    try:
        out = pool.map(fn, items)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


def _gen_slice(spec):
    from synth import generate
    c = generate(spec)
    return c.indptr, c.indices, c.data, c.mu


def run_slices(args) -> None:
    """Batched time slices: 64 independent corpora of uneven sizes, each with
    its own whitening, K and Phi, stepped per batch index.  Timed four ways
    over whole passes: one tlda_whiten_cp_step call per slice batch; one
    multi-slice plan step per batch index; the same captured in a HIP graph;
    and the graph after the autotuner picked each plan's launch shape."""
    import numpy as np

    from synth import Corpus, init_phi, iter_batches, slice_specs
    specs = slice_specs(scale=args.slice_scale)
    t = time.time()
    parts = _fork_map(_gen_slice, specs, args.gen_workers)
    corpora = [Corpus(sp, ip, ix, dt, mu, sp.alpha) for sp, (ip, ix, dt, mu) in zip(specs, parts)]
    del parts
    n_docs = sum(c.n_docs for c in corpora)
    log(f"[bench] generated {len(corpora)} slices, {n_docs} docs "
        f"({min(c.n_docs for c in corpora)} .. {max(c.n_docs for c in corpora)}) "
        f"in {time.time() - t:.1f}s")
    import torch

    from paper_2511_07809_amd import tlda as tl
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t = time.time()
    ctxs, dev, phis0 = [], [], []
    for c in corpora:
        sp = c.spec
        ctx = tl.tlda_create(sp.V, sp.K, sp.K, sp.alpha0, 0.0, bf16=True, eig_iters=30,
                             stream=stream)
        bs = [tl.CsrBatch.from_numpy(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
        torch.cuda.synchronize()
        for b in bs:
            tl.tlda_update_moments(ctx, b)
        tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W | tl.TLDA_RELEASE)
        ctxs.append(ctx)
        dev.append(bs)
        phis0.append(init_phi(sp.K, sp.K, 1).astype(np.float32))
    log(f"[bench] moments, whitening refresh and release of {len(ctxs)} slices in "
        f"{time.time() - t:.1f}s")
    n_idx = max(len(b) for b in dev)
    beta = 1e-3
    Ps = [torch.from_numpy(p).cuda() for p in phis0]
    nk = torch.zeros(len(ctxs), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    plans, members = [], []
    for i in range(n_idx):
        idx = [s for s in range(len(ctxs)) if len(dev[s]) > i]
        members.append(idx)
        plans.append(tl.tlda_multi_create([ctxs[s] for s in idx], [dev[s][i] for s in idx],
                                          [Ps[s] for s in idx], [beta] * len(idx),
                                          nk[:len(idx)]))

    def reset():
        torch.cuda.synchronize()
        for P, p0 in zip(Ps, phis0):
            P.copy_(torch.from_numpy(p0).cuda())
        torch.cuda.synchronize()

    def per_slice_pass():
        for s, ctx in enumerate(ctxs):
            for b in dev[s]:
                tl.tlda_whiten_cp_step(ctx, b, beta, Ps[s])

    def multi_pass():
        for p in plans:
            tl.tlda_multi_step(p)

    def timed(fn, passes):
        reset()
        fn()                                  # warm-up pass
        stream.synchronize()
        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(passes):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / passes

    passes = max(1, args.steps // 8)
    res_ms = {"per_slice_calls": timed(per_slice_pass, passes), "multi_eager": timed(multi_pass, passes)}
    graph = tl.tlda_graph_capture(plans)
    res_ms["multi_graph"] = timed(lambda: tl.tlda_graph_launch(graph), passes)
    reset()
    default_tiles = [tl.tlda_multi_get_tile(p) for p in plans]
    tuned = [tl.tlda_multi_autotune(p, 3) for p in plans]
    tuned_tiles = [tl.tlda_multi_get_tile(p) for p in plans]
    graph_t = tl.tlda_graph_capture(plans)
    res_ms["multi_graph_autotuned"] = timed(lambda: tl.tlda_graph_launch(graph_t), passes)
    for k, v in res_ms.items():
        log(f"[bench] {k}: {v:.3f} ms per pass, {n_docs / (v / 1e3):.4g} docs/s")
    best = min(res_ms, key=res_ms.get)
    ms = res_ms[best]
    # agreement of the batched path with the per-slice calls after a few passes
    reset()
    for _ in range(args.fit_passes):
        tl.tlda_graph_launch(graph_t)
    stream.synchronize()
    multi_phi = [P.cpu().numpy().copy() for P in Ps]
    reset()
    for _ in range(args.fit_passes):
        per_slice_pass()
    stream.synchronize()
    diff = max(float(np.linalg.norm(P.cpu().numpy() - m) / max(np.linalg.norm(m), 1e-30))
               for P, m in zip(Ps, multi_phi))
    nnz = sum(c.nnz for c in corpora)
    # CSR of every batch, plus each slice's BF16 whitening copy once per batch
    alg_bytes = 4 * (n_docs + sum(len(b) for b in dev)) + 8 * nnz + \
        sum(len(dev[s]) * 2 * corpora[s].spec.V * corpora[s].spec.K for s in range(len(dev)))
    ach = alg_bytes / (ms / 1e3) / 1e9
    out = {
        "metric": "docs/sec (whiten+CP step) over 64 batched time slices, one step launch "
                  "per batch index, the pass in one graph",
        "value": n_docs / (ms / 1e3), "unit": "docs/s", "n_gpus": 1, "steps": passes,
        "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"{len(ctxs)} slices sharing V=20000, {n_docs} docs, sizes "
                               f"lognormal (median 150000, sigma 1, clip 1e4..2e6) x "
                               f"{args.slice_scale:g}, K in {{10, 20, 50}}, batch 131072",
                   "path": best, "batch_indices": n_idx},
        "roofline": {"kernel": "k_cp_bf16_multi + k_cp_finish_multi (whole pass)",
                     "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_pass": alg_bytes},
        "breakdown": {**{f"{k}_ms_per_pass": v for k, v in res_ms.items()},
                      **{f"{k}_docs_per_s": n_docs / (v / 1e3) for k, v in res_ms.items()},
                      "autotuned_total_blocks": tuned,
                      "default_tile_shapes": [f"{r}x{w}" for r, w in default_tiles],
                      "autotuned_tile_shapes": [f"{r}x{w}" for r, w in tuned_tiles],
                      # one step kernel and one finish kernel per batch index;
                      # the graph path submits the whole pass with one host call
                      "kernel_launches_per_pass": 2 * n_idx,
                      "host_calls_per_pass": {"per_slice_calls": sum(len(b) for b in dev),
                                              "multi_eager": n_idx, "multi_graph": 1,
                                              "multi_graph_autotuned": 1},
                      "multi_vs_per_slice_phi_rel_diff": diff,
                      "passes_compared": args.fit_passes},
    }
    print(json.dumps(out), flush=True)


def make_corpus(spec, n_docs: int, workers: int):
    """The workload's corpus, generated by forked workers: call it before the
    process first uses the GPU."""
    from synth import generate
    t = time.time()
    corpus = generate(spec, n_docs=n_docs or None, workers=workers)
    log(f"[bench] generated {spec.name}: {corpus.n_docs} docs, {corpus.nnz} nnz in "
        f"{time.time() - t:.1f}s")
    return corpus


def measure(tl, spec, args, precision: str, corpus, stream) -> dict:
    """One workload: moment pass and refresh over `corpus`, the timed steps of
    both precisions (eager and graph), the roofline of the main precision's
    kernel and the topic error of both precisions after the same passes."""
    import numpy as np
    import torch

    from synth import init_phi, iter_batches

    D = K = spec.K
    batches = list(iter_batches(corpus))
    bf16 = precision == "bf16"
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, bf16=bf16, eig_iters=60, stream=stream)
    dev = [tl.CsrBatch.from_numpy(rp, ci, va, first_doc=int(i * spec.batch))
           for i, (rp, ci, va, _) in enumerate(batches)]
    torch.cuda.synchronize()

    # ---- moment pass (a1) and refresh, timed on the context's stream ----
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for b in dev:
        tl.tlda_update_moments(ctx, b)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_ref = time.perf_counter()
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    refresh_ms = (time.perf_counter() - t_ref) * 1e3
    moments_ms = ev[0].elapsed_time(ev[1])
    log(f"[bench] {spec.name} moment pass {moments_ms:.2f} ms, refresh {refresh_ms:.1f} ms")
    # free the V x V accumulator (20 GB at V = 50 000) now that W exists
    tl.tlda_update_moments(ctx, None, tl.TLDA_RELEASE)
    # the other precision on the same whitening, for the side-by-side figures
    W, _, m = tl.tlda_get_whitening(ctx)
    other = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, bf16=not bf16, stream=stream)
    tl.tlda_set_whitening(other, W, m)

    # ---- CP steps (a2 + a3) ----
    beta = args.beta if args.beta is not None else (0.03 if spec.name == "c1" else 1e-3)
    Xbuf = torch.empty((max(b.n_rows for b in dev), D), dtype=torch.float32, device="cuda")
    nk = torch.empty(1, dtype=torch.int32, device="cuda")
    fused = args.path == "fused"

    def stage_format_for(prec):
        if args.stage_format != "auto":
            return args.stage_format
        return "u16" if prec == "bf16" and spec.V <= 65536 else "f32"
    stage_format = stage_format_for(precision)
    if args.streamed:
        hosts = {}
        if "u16" in (stage_format_for("bf16"), stage_format_for("fp32")):
            hosts["u16"] = [tl.CsrBatchU16(rp, ci, va) for rp, ci, va, _ in batches]
        if "f32" in (stage_format_for("bf16"), stage_format_for("fp32")):
            hosts["f32"] = [tl.CsrBatch.from_numpy(rp, ci, va, pin=True)
                            for rp, ci, va, _ in batches]

        def make_batch_for(cx):
            fmt = stage_format_for("bf16" if cx is (ctx if bf16 else other) else "fp32")
            host = hosts[fmt]
            stage = tl.tlda_stage_batch_u16 if fmt == "u16" else tl.tlda_stage_batch
            staged = {}

            def batch_for(i):
                # stage batch i+1 before computing batch i, so the copy overlaps the compute
                if i not in staged:
                    staged.clear()
                    staged[i] = stage(cx, host[i % len(host)], i % 2)
                staged[i + 1] = stage(cx, host[(i + 1) % len(host)], (i + 1) % 2)
                return staged.pop(i)
            return batch_for
    else:
        def make_batch_for(cx):
            return lambda i: dev[i % len(dev)]

    other_name = "fp32" if bf16 else "bf16"
    runs = {}
    for name, cx in ((precision, ctx), (other_name, other)):
        Phi = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
        r = run_steps(tl, cx, make_batch_for(cx), fused, beta, Phi, Xbuf, nk, args.steps,
                      args.warmup, stream)
        r["docs_per_s"] = r["docs"] / (r["total_ms"] / 1e3)
        runs[name] = r
        km = r["kern_ms"].mean(axis=0) * 1e3
        log(f"[bench] {spec.name} {name} {args.path}: {args.steps} steps {r['total_ms']:.3f} ms "
            f"(wall {r['wall_ms']:.1f} ms), step {r['step_ms'].mean() * 1e3:.1f} us, main "
            f"kernel(s) {' + '.join(f'{x:.1f}' for x in km)} us, {r['docs_per_s']:.4g} docs/s")
    # the same K steps as one captured HIP graph (no host launch gaps); the
    # kernels and their launch shapes are those of the eager steps above
    graph_runs = {}
    if fused and not args.streamed:
        for name, cx in ((precision, ctx), (other_name, other)):
            steps_b = [dev[(args.warmup + i) % len(dev)] for i in range(args.steps)]
            Phi = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
            torch.cuda.synchronize()
            try:
                g = tl.tlda_graph_capture_steps(cx, steps_b, beta, Phi)
            except tl.TldaError as err:      # e.g. FP32 steps above the fused shapes
                log(f"[bench] {name}: steps not captured ({err}); eager only")
                continue
            for _ in range(GRAPH_WARM_REPLAYS):      # untimed replays
                tl.tlda_graph_launch(g)
            torch.cuda.synchronize()
            # GRAPH_REPLAYS timed replays of the K steps, each bracketed by
            # events and a synchronisation; the median replay gives the rate
            reps = []
            for _ in range(GRAPH_REPLAYS):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                tl.tlda_graph_launch(g)
                e1.record(stream)
                torch.cuda.synchronize()
                reps.append(e0.elapsed_time(e1))
            ms = float(np.median(reps))
            graph_runs[name] = {"total_ms": ms, "replay_ms": reps,
                                "docs_per_s": sum(b.n_rows for b in steps_b) / (ms / 1e3)}
            log(f"[bench] {spec.name} {name} graph of {args.steps} steps: median {ms:.3f} ms of "
                f"{GRAPH_REPLAYS} replays ({', '.join(f'{x:.3f}' for x in reps)}), "
                f"{graph_runs[name]['docs_per_s']:.4g} docs/s")
            del g
    main_run = runs[precision]
    K_steps = args.steps

    # ---- roofline of the dominant kernel, on its own launch duration ----
    docs, nnz_tot = main_run["docs"], main_run["nnz"]
    rows_per = docs / K_steps
    csr_bytes = (4 * (docs + K_steps) + 8 * nnz_tot) / K_steps      # row_ptr, col_idx, val
    w_elem = 2 if bf16 else 4
    w_bytes = w_elem * spec.V * D + 4 * D                             # W copy and W^T M1, once
    cp_flops = rows_per * (4.0 * D * K + K)
    mm_peak = BF16_MFMA_PEAK_TFLOPS if bf16 else FP32_VALU_PEAK_TFLOPS
    kern_us = main_run["kern_ms"].mean(axis=0) * 1e3
    if fused:
        t_k = kern_us[0] / 1e6
        if bf16:
            name, key = "k_cp_bf16 (fused mode)", "k_cp_bf16/fused"
        else:
            name = key = fp32_fused_kernel(D, K)
        hbm_frac = (csr_bytes + w_bytes) / t_k / 1e9 / HBM_PEAK_GBS
        mm_frac = cp_flops / t_k / 1e12 / mm_peak
        if hbm_frac >= mm_frac:
            ach = (csr_bytes + w_bytes) / t_k / 1e9
            roof = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
        else:
            ach = cp_flops / t_k / 1e12
            roof = {"kernel": name, "bound": "mfma", "achieved": ach, "peak": mm_peak,
                    "unit": "TFLOP/s", "frac": ach / mm_peak}
        # beside it: the whitening-row gathers, one row of D elements of the
        # whitening copy per nonzero, served by the caches
        gather_bytes = nnz_tot / K_steps * D * w_elem
        roof.update({"traffic": measured_traffic(key, spec.name),
                     "algorithmic_bytes": csr_bytes + w_bytes, "algorithmic_flops": cp_flops,
                     "hbm_frac": hbm_frac, "mfma_frac": mm_frac,
                     "gather_bytes": gather_bytes, "gather_TBps": gather_bytes / t_k / 1e12,
                     "avg_launch_us": float(kern_us[0])})
    else:
        wh_bytes = csr_bytes + 4 * D * rows_per + w_bytes
        wh_s, cp_s = kern_us[0] / 1e6, kern_us[1] / 1e6
        if wh_s >= cp_s:
            name = "k_cp_bf16 (whitening mode)" if bf16 else "k_whiten"
            key = "k_cp_bf16/whiten" if bf16 else "k_whiten"
            ach = wh_bytes / wh_s / 1e9
            roof = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": measured_traffic(key, spec.name),
                    "algorithmic_bytes": wh_bytes, "avg_launch_us": float(kern_us[0])}
        else:
            name = "k_cp_bf16 (from-X mode)" if bf16 else "k_cp_reduce_mfma"
            key = "k_cp_bf16/from_x" if bf16 else "k_cp_reduce_mfma"
            ach = cp_flops / cp_s / 1e12
            roof = {"kernel": name, "bound": "mfma", "achieved": ach, "peak": mm_peak,
                    "unit": "TFLOP/s", "frac": ach / mm_peak,
                    "traffic": measured_traffic(key, spec.name),
                    "algorithmic_flops": cp_flops, "avg_launch_us": float(kern_us[1])}

    # ---- topic-recovery error of both precisions after the same passes ----
    fit_beta = args.fit_beta
    if fit_beta is None:
        fit_beta = {"c1": 0.03, "c2": 0.01}.get(spec.name, 1e-3)
    acc = {"passes": args.fit_passes, "beta": fit_beta}
    mus = {}
    for name, cx in ((precision, ctx), (other_name, other)):
        Phi = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
        for _ in range(args.fit_passes):
            for b in dev:
                tl.tlda_whiten_cp_step(cx, b, fit_beta, Phi)
        acc[f"{name}_topic_l1_to_planted"], mus[name] = topic_error(tl, cx, Phi, corpus.mu)
    acc["fp32_vs_bf16_topic_l1"] = float(np.abs(mus["fp32"] - mus["bf16"]).sum(axis=0).mean())
    log(f"[bench] {spec.name} topic error after {args.fit_passes} passes: {acc}")
    return {"corpus": corpus, "batches": batches, "runs": runs, "graph_runs": graph_runs,
            "roof": roof, "acc": acc, "moments_ms": moments_ms, "refresh_ms": refresh_ms,
            "W": W, "m": m, "stage_format": stage_format, "beta": beta, "kern_us": kern_us,
            "other_name": other_name}


def run_full_stream(args) -> None:
    """The workload as configured end to end: every document of the corpus
    (20 000 000 at the streaming scale) streamed from pinned host memory in
    its batches, each staged on the copy stream (tlda_stage_batch_u16, or
    tlda_stage_batch with --stage-format f32) while the previous batch
    computes: one moment pass, the whitening refresh, then --cp-passes passes
    of fused CP steps in BF16 and then in FP32 from the same start on the same
    whitening.  Reports the PCIe-inclusive rate of the CP passes and the topic
    error after them; `value` is the BF16 rate (the configured precision)."""
    import numpy as np
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS, generate, init_phi, iter_batches
    spec = SPECS[args.workload]
    n_docs = args.docs or spec.N
    D = K = spec.K
    t = time.time()
    corpus = generate(spec, n_docs=n_docs, workers=args.gen_workers)
    batches = list(iter_batches(corpus))
    log(f"[bench] generated {spec.name}: {corpus.n_docs} docs, {corpus.nnz} nnz, "
        f"{len(batches)} batches in {time.time() - t:.1f}s")
    fmt = args.stage_format if args.stage_format != "auto" else (
        "u16" if spec.V <= 65536 and float(corpus.data.max()) <= 65535 else "f32")
    t = time.time()
    if fmt == "u16":
        hosts = [tl.CsrBatchU16(rp, ci, va, first_doc=int(fd)) for rp, ci, va, fd in batches]
        stage = tl.tlda_stage_batch_u16
    else:
        hosts = [tl.CsrBatch.from_numpy(rp, ci, va, pin=True, first_doc=int(fd))
                 for rp, ci, va, fd in batches]
        stage = tl.tlda_stage_batch
    host_mb = sum(h.row_ptr.numel() * 4 + h.col_idx.numel() * h.col_idx.element_size()
                  + h.val.numel() * h.val.element_size() for h in hosts) / 1e6
    log(f"[bench] pinned {len(hosts)} host batches ({fmt}, {host_mb:.0f} MB) in "
        f"{time.time() - t:.1f}s")
    del batches
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    nb = len(hosts)

    def stream_pass(cx, fn):
        """Stage batch i + 1 before computing batch i (two slots)."""
        cur = stage(cx, hosts[0], 0)
        for i in range(nb):
            nxt = stage(cx, hosts[i + 1], (i + 1) % 2) if i + 1 < nb else None
            fn(cur)
            cur = nxt

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, bf16=True, eig_iters=60, stream=stream)
    moments_ms = timed(lambda: stream_pass(ctx, lambda b: tl.tlda_update_moments(ctx, b)))
    t_ref = time.perf_counter()
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    torch.cuda.synchronize()
    refresh_ms = (time.perf_counter() - t_ref) * 1e3
    N, skipped, _ = tl.tlda_get_stats(ctx)     # (the release below clears them)
    tl.tlda_update_moments(ctx, None, tl.TLDA_RELEASE)
    log(f"[bench] streamed moment pass {moments_ms:.1f} ms ({n_docs / (moments_ms / 1e3):.4g} "
        f"docs/s), refresh {refresh_ms:.1f} ms; N = {N}, dropped {skipped}")
    W, _, m = tl.tlda_get_whitening(ctx)
    fp32 = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, stream=stream)
    tl.tlda_set_whitening(fp32, W, m)
    beta = args.beta if args.beta is not None else 1e-3
    phi0 = init_phi(D, K, 1).astype(np.float32)
    res = {}
    for name, cx in (("bf16", ctx), ("fp32", fp32)):
        Phi = torch.from_numpy(phi0).cuda()
        torch.cuda.synchronize()
        per_pass = [timed(lambda: stream_pass(cx, lambda b: tl.tlda_whiten_cp_step(cx, b, beta,
                                                                                   Phi)))
                    for _ in range(args.cp_passes)]
        total = float(sum(per_pass))
        err, _ = topic_error(tl, cx, Phi, corpus.mu)
        res[name] = {"docs_per_s": args.cp_passes * n_docs / (total / 1e3),
                     "pass_ms": per_pass, "topic_l1_to_planted": err}
        log(f"[bench] {name}: {args.cp_passes} streamed passes {total:.1f} ms "
            f"({', '.join(f'{x:.1f}' for x in per_pass)}), "
            f"{res[name]['docs_per_s']:.4g} docs/s, topic error {err:.4f}")
    steps = args.cp_passes * nb
    out = {
        "metric": f"docs/sec over {args.cp_passes} CP passes of the whole corpus streamed from "
                  "pinned host memory (PCIe-inclusive)",
        "value": res["bf16"]["docs_per_s"], "unit": "docs/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": sum(res["bf16"]["pass_ms"]) / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: V={spec.V}, K=D={K}, alpha0={spec.alpha0}, "
                               f"{n_docs} docs in {nb} batches of up to {spec.batch}, streamed "
                               f"from pinned host memory ({fmt} staging), {args.cp_passes} CP "
                               "passes", "mode": "full_stream", "beta": beta},
        "roofline": None,
        "breakdown": {"moment_pass_ms": moments_ms, "refresh_ms": refresh_ms,
                      "n_kept": int(N), "n_dropped": int(skipped), "host_batch_mb": host_mb,
                      "bf16": res["bf16"], "fp32": res["fp32"]},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.warmup is None:
        args.warmup = 1 if args.online else 64
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c5":
        run_encoder(args)
        return
    if args.workload == "c4":
        run_slices(args)
        return
    if args.estimator == "classic":
        run_classic(args)
        return
    if args.online:
        run_online(args)
        return
    if args.full_stream:
        run_full_stream(args)
        return
    import torch

    from paper_2511_07809_amd import tlda as tl
    from synth import SPECS

    spec = SPECS[args.workload]
    n_docs = args.docs or (16 * spec.batch if spec.name == "c3" else 0)
    with_c2 = spec.name == "c3" and not args.no_c2 and not args.streamed and not args.docs
    # corpora first: their generation forks worker processes, which must
    # happen before this process touches the GPU
    corpus_main = make_corpus(spec, n_docs, args.gen_workers)
    corpus_c2 = make_corpus(SPECS["c2"], 0, args.gen_workers) if with_c2 else None
    torch.cuda.set_device(0)
    # a stream of its own (default priority): the null stream cannot be captured
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    res = measure(tl, spec, args, args.precision, corpus_main, stream)
    del corpus_main
    corpus, runs, graph_runs = res["corpus"], res["runs"], res["graph_runs"]
    main_run, main_graph = runs[args.precision], graph_runs.get(args.precision)
    other_name = res["other_name"]
    K = spec.K
    mom_docs_s = corpus.n_docs / (res["moments_ms"] / 1e3)
    bf16 = args.precision == "bf16"
    out = {
        "metric": "docs/sec (whiten+CP step) at fixed topic-recovery error; % HBM roofline",
        "value": (main_graph or main_run)["docs_per_s"], "unit": "docs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (main_graph or main_run)["total_ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if bf16 else "f32", "data": "synthetic",
        "config": {"workload": f"{spec.name}: V={spec.V}, K=D={K}, alpha0={spec.alpha0}, "
                               f"{corpus.n_docs} docs ({len(res['batches'])} distinct batches of "
                               f"{spec.batch}) of length 1+Poisson({spec.doc_len_lambda:g}), "
                               + ("streamed from pinned host memory" if args.streamed
                                  else "resident in HBM"),
                   "streamed": bool(args.streamed), "precision": args.precision,
                   "stage_format": res["stage_format"] if args.streamed else None,
                   "global_batch": spec.batch, "beta": res["beta"], "path": args.path,
                   "launch": "hip_graph" if main_graph else "eager"},
        "roofline": res["roof"],
        "breakdown": {"path": args.path,
                      "eager_docs_per_s": main_run["docs_per_s"],
                      "graph_docs_per_s": main_graph["docs_per_s"] if main_graph else None,
                      "graph_replay_ms": main_graph["replay_ms"] if main_graph else None,
                      f"{other_name}_graph_docs_per_s":
                          graph_runs[other_name]["docs_per_s"] if other_name in graph_runs else None,
                      "step_us": float(main_run["step_ms"].mean()) * 1e3,
                      "main_kernel_us": [float(x) for x in res["kern_us"]],
                      f"{other_name}_docs_per_s": runs[other_name]["docs_per_s"],
                      f"{other_name}_step_us": float(runs[other_name]["step_ms"].mean()) * 1e3,
                      f"{other_name}_main_kernel_us":
                          [float(x) for x in runs[other_name]["kern_ms"].mean(axis=0) * 1e3],
                      "moment_pass_ms": res["moments_ms"], "moments_docs_per_s": mom_docs_s,
                      "refresh_ms": res["refresh_ms"]},
        "accuracy": res["acc"],
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on one batch (single-thread and all cores)")
        rp, ci, va, _ = res["batches"][0]
        out["cpu_baseline"] = cpu_baseline(spec, (rp, ci, va), res["W"], res["m"], args.cpu_reps)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.4g} docs/s "
            f"({out['cpu_baseline']['cores']} threads), single thread "
            f"{out['cpu_baseline']['single_thread_docs_per_s']:.4g}")
    if with_c2:
        del res
        c2 = measure(tl, SPECS["c2"], args, args.precision, corpus_c2, stream)
        out["breakdown"]["c2"] = {
            "workload": f"c2: V=20000, K=D=50, {c2['corpus'].n_docs} docs, batch "
                        f"{SPECS['c2'].batch}, resident in HBM",
            **{f"{n}_graph_docs_per_s": g["docs_per_s"] for n, g in c2["graph_runs"].items()},
            **{f"{n}_main_kernel_us": float(r["kern_ms"].mean() * 1e3)
               for n, r in c2["runs"].items()},
            "roofline": {k: c2["roof"][k] for k in ("kernel", "bound", "frac", "hbm_frac",
                                                   "mfma_frac", "avg_launch_us")},
            "accuracy": c2["acc"]}
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
