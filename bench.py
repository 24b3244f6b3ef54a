"""Throughput of the CoR-UTV hot path on one MI355X.

Default workload: A = 20000 x 10000 = U diag(sigma) V^T with U, V random
orthonormal (QR of seeded Gaussians) and sigma_i = i^-1.5; k = 200, p = 20
(l = 220), q = 2.  One step is one whole decomposition (Omega, 2q+2 passes
over A with CholeskyQR after each, M = R2^T, QRCP, U and V), replayed from a
captured HIP graph of the plan.  The decomposition runs with its passes in
FP64 (the line's value: the paper's arithmetic), FP32, BF16 and FP8 E4M3 with
per-column scales; every result is checked against the oracle's stored result
for the same matrix and test matrix (at fixed error), and every format
reports its own throughput, error ratio and pass roofline.

Prints one JSON line: decompositions/s, p50/p99 step latency, the roofline of
the dominant kernel (the passes over A) from HIP events around every pass
launch of eager runs on the plan's stream, and the FP64 CPU oracle timed end
to end on two row blocks of the same matrix.
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

PEAKS = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp8": 5000.0,  # TFLOP/s
}

WORKLOADS = {
    # default: the 20000 x 10000 workload in every pass format (value = FP64)
    "c3": dict(desc="20000x10000, U, V random orthonormal, sigma_i=i^-1.5; k=200, l=220, q=2; "
                    "passes in FP64 (value), FP32, BF16 and FP8 E4M3 with column scales"),
    "c2": dict(m=8000, n=8000, rank=500, spectrum="exp40", k=100, p=10, q=2, prec="f32", seed=202,
               desc="8000x8000 FP32, rank-500 Haar factors, sigma_i=exp(-i/40); k=100, l=110, q=2"),
    "c3bf16": dict(m=20000, n=10000, rank=10000, spectrum="pow15", k=200, p=20, q=2, prec="bf16",
                   seed=303, desc="20000x10000 BF16, sigma_i=i^-1.5; k=200, l=220, q=2"),
    "c1": dict(m=1000, n=1000, rank=1000, spectrum="c1", k=10, p=5, q=1, prec="f64", seed=101,
               noise=1e-6, desc="1000x1000 FP64, sigma 1 (i<=10) then 1e-3*0.9^(i-10); k=10, l=15, q=1"),
    # robust PCA by ALM-CoRUTV on the synthetic L + S matrix of the recovery
    # experiment (Table I's largest shape; l = k + 64, the largest l supported)
    "rpca": dict(n=4000, rank=200, frac=0.05, k=200, p=64, q=1, seed=606, cpu_iters=1,
                 desc="robust PCA, M = L + S 4000x4000, rank(L)=200, 5% +-80 outliers; "
                      "ALM-CoRUTV k=200, l=264, q=1, FP64"),
    # the tall robust-PCA request shape with the fused power step
    "tall": dict(m=76800, n=2000, rank=5, frac=0.05, k=5, p=8, q=2, seed=707,
                 desc="76800x2000 FP32 (rank 5 + 5% +-80 outliers), k=5, l=13, q=2; fused power "
                      "step (q + 2 = 4 reads of A) against the two-pass step (2q + 2 = 6)"),
    # A in pinned host memory, streamed in panels for every pass
    "host": dict(m=200000, n=1000, rank=5, frac=0.05, k=5, p=8, q=2, seed=808, panel_rows=32768,
                 desc="200000x1000 FP32 in pinned host memory (rank 5 + 5% +-80 outliers), k=5, "
                      "l=13, q=2, panels of 32768 rows; fused power step (q + 2 = 4 streams of A) "
                      "and two-pass step (6 streams)"),
    # many independent problems in one batched plan (BF16 passes)
    "c4batched": dict(count=512, seed=404, prec="bf16",
                      desc="512 problems, m,n ~ U{256..4096}, k ~ U{8..64}, l=k+8, q=1, "
                           "sigma_i=exp(-i/k), BF16 passes, one batched plan"),
    # open-loop served requests: BF16-served vs plain sequential FP32
    "c5served": dict(count=160, seed=505, pool=16,
                     desc="Poisson requests, m,n log-uniform [512,16384], k ~ U{16..256}, p=8, "
                          "q ~ U{0,1,2}, 10% robust-PCA 76800x2000; FP32 inputs served in BF16 "
                          "vs plain sequential FP32"),
}


def source_hash(fname="k_sketch.hip"):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1810_07323_amd", "csrc", fname), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def make_input(w, dev):
    import numpy as np
    import torch

    import inputs as I

    r = w["rank"]
    sig = I.spectrum(w["spectrum"], r)
    a64, sig = I.lowrank(w["m"], w["n"], sig, w["seed"], noise=w.get("noise", 0.0),
                         backend="torch", device=dev)
    return a64, np.asarray(sig)


def bench_batched(args, w, cu, torch, np):
    """Decompositions/s of one batched plan over many independent problems."""
    import inputs as I

    dev = torch.device("cuda:0")
    specs = I.batched_problems(w["count"], w["seed"])
    mats, probs, outs, sigs = [], [], [], []
    for s in specs:
        sig = I.spectrum("expk", s["rank"], s["k"])
        a64, _ = I.lowrank(s["m"], s["n"], sig, s["seed"], backend="torch", device=dev)
        A = a64.to(torch.bfloat16).contiguous()
        del a64
        l = s["k"] + s["p"]
        o = (torch.empty((s["m"], l), dtype=torch.float64, device=dev),
             torch.empty((l, l), dtype=torch.float64, device=dev),
             torch.empty((s["n"], l), dtype=torch.float64, device=dev),
             torch.empty((l,), dtype=torch.int32, device=dev))
        probs.append(cu.make_problem(A, s["k"], s["p"], s["q"], s["seed"], *o))
        mats.append(A)
        outs.append(o)
        sigs.append(sig)
    stream = torch.cuda.Stream()
    st, plan = cu.cor_plan_create(probs, cu.cor_opts(0, 0))
    cu.check(st, "plan_create")
    with torch.cuda.stream(stream):
        if not args.no_graph:
            cu.check(cu.cor_plan_capture(plan, stream), "plan_capture")
        for _ in range(args.warmup):
            cu.check(cu.cor_plan_run(plan, stream), "plan_run")
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            cu.check(cu.cor_plan_run(plan, stream), "plan_run")
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # roofline of the passes: an eager plan over the same problems
        st2, plan2 = cu.cor_plan_create(probs, cu.cor_opts(0, 0))
        cu.check(st2, "plan_create")
        cu.cor_profile_enable(True)
        cu.cor_profile_read()
        for _ in range(min(args.steps, 5)):
            cu.check(cu.cor_plan_run(plan2, stream), "plan_run")
        torch.cuda.synchronize()
        prof = cu.cor_profile_read()
        cu.cor_profile_enable(False)
        cu.cor_plan_destroy(plan2)
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    elapsed = t1 - t0
    # accuracy of a sample of the timed results against their optimum
    worst = 0.0
    for j in range(0, len(specs), max(1, len(specs) // 16)):
        s, (U, T, V, _) = specs[j], outs[j]
        a = mats[j].double()
        err = float(torch.linalg.norm(a - (U @ T) @ V.T) / torch.linalg.norm(a))
        s2 = sigs[j] ** 2
        l = s["k"] + s["p"]
        opt = float(np.sqrt(s2[l:].sum() / s2.sum())) if len(s2) > l else 0.0
        worst = max(worst, err / max(opt, 1e-300) if opt > 0 else err)
        del a
    launches = max(1, prof["launches"])
    avg_s = prof["ms"] / launches / 1e3
    achieved = prof["bytes"] / launches / avg_s / 1e9
    cu.cor_plan_destroy(plan)
    return {
        "metric": "CoR-UTV decompositions/s (roofline of the passes over A; p50/p99 latency)",
        "value": round(len(specs) * args.steps / elapsed, 3),
        "unit": "decomps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": args.workload + ": " + w["desc"], "problems": len(specs),
                   "graph": not args.no_graph},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4)},
        "accuracy": {"worst_err_l_over_opt_sampled": worst},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAKS["hbm_GBs"],
                     "unit": "GB/s", "frac": round(achieved / PEAKS["hbm_GBs"], 4),
                     "traffic": None, "kernel": "k_sketch (passes over A, all problems)",
                     "avg_launch_us": round(avg_s * 1e6, 2)},
        "cpu_baseline": None,
    }


def bench_served(args, w, cu, torch, np):
    """Open-loop served requests (FP32 inputs converted and served in BF16)
    against the plain path (each FP32 request alone, one after another)."""
    import inputs as I

    dev = torch.device("cuda:0")
    reqs = I.served_requests(w["count"], w["seed"], rate=1.0, pool=w["pool"])
    # matrices: a pool of decaying-spectrum FP32 matrices and one robust-PCA input
    pool = {}
    for r in reqs:
        if r["kind"] == "decay" and r["pool"] not in pool:
            j = r["pool"]
            m, n = r["m"], r["n"]
            kj = 16 + (j * 37) % 241
            rank = min(m, n, 4 * (kj + 8))
            sig = I.spectrum("expk", rank, kj)
            a64, _ = I.lowrank(m, n, sig, w["seed"] * 100 + j, backend="torch", device=dev)
            pool[j] = a64.float().contiguous()
            del a64
    rp = None
    if any(r["kind"] == "rpca" for r in reqs):
        g = torch.Generator(device=dev).manual_seed(w["seed"])
        g1 = torch.randn(76800, 5, generator=g, device=dev)
        g2 = torch.randn(2000, 5, generator=g, device=dev)
        rp = g1 @ g2.T
        cnt = int(round(0.05 * rp.numel()))
        pos = torch.randperm(rp.numel(), generator=g, device=dev)[:cnt]
        sgn = torch.where(torch.rand(cnt, generator=g, device=dev) < 0.5, -80.0, 80.0)
        rp.view(-1)[pos] += sgn
        rp = rp.contiguous()

    def mat(r):
        return rp if r["kind"] == "rpca" else pool[r["pool"]]

    def outputs(r):
        l = r["k"] + r["p"]
        return (torch.empty((r["m"], l), dtype=torch.float64, device=dev),
                torch.empty((l, l), dtype=torch.float64, device=dev),
                torch.empty((r["n"], l), dtype=torch.float64, device=dev),
                torch.empty((l,), dtype=torch.int32, device=dev))

    opts = cu.cor_opts(1, 0)  # report: each result carries its error
    # plain path: FP32, one request after another, each from a plan created
    # (workspace allocated, descriptors uploaded) before the timed loop, so the
    # comparison measures batching rather than allocation
    plans = []
    for r in reqs:
        o = outputs(r)
        st, plan = cu.cor_plan_create(
            [cu.make_problem(mat(r), r["k"], r["p"], r["q"], r["seed"], *o)], opts)
        cu.check(st, "plain plan")
        plans.append((plan, o))
    for plan, _ in plans[:2]:  # warm the code paths
        cu.check(cu.cor_plan_run(plan), "plain warmup")
        cu.check(cu.cor_plan_info(plan, 1)[0], "plain warmup")
    torch.cuda.synchronize()
    plain_err, plain_lat = [], []
    t0 = time.perf_counter()
    for plan, _ in plans:
        ts = time.perf_counter()
        cu.check(cu.cor_plan_run(plan), "plain")
        st, infos = cu.cor_plan_info(plan, 1)  # waits for the request
        cu.check(st, "plain info")
        plain_lat.append((time.perf_counter() - ts) * 1e3)
        plain_err.append(infos[0].err_l)
    torch.cuda.synchronize()
    plain_rate = len(reqs) / (time.perf_counter() - t0)
    for plan, _ in plans:
        cu.cor_plan_destroy(plan)
    del plans

    def serve(rate):
        st, srv = cu.cor_server_create(hbm_budget=0, max_slots=0, convert_f32_to=cu.COR_BF16)
        cu.check(st, "server_create")
        keep, tickets = [], []
        try:
            start = time.perf_counter()
            for r in reqs:
                due = start + (r["t"] / rate if rate else 0.0)
                now = time.perf_counter()
                if due > now:
                    time.sleep(due - now)
                o = outputs(r)
                pr = cu.make_problem(mat(r), r["k"], r["p"], r["q"], r["seed"], *o)
                st, t = cu.cor_server_submit(srv, pr, opts)
                cu.check(st, "submit")
                keep.append((pr, o))
                tickets.append(t)
            errs = []
            for t in tickets:
                st, info = cu.cor_server_wait(srv, t)
                cu.check(st, "wait")
                errs.append(info.err_l)
            st, stats = cu.cor_server_stats_get(srv)
            cu.check(st, "stats")
            return stats.as_dict(), errs
        finally:
            cu.check(cu.cor_server_destroy(srv), "destroy")

    sat, errs = serve(0.0)  # every request at once: saturation throughput
    lam = 0.8 * sat["decomps_per_s"]
    open_loop, errs2 = serve(lam)  # Poisson arrivals at 0.8 x saturation
    # Requests whose FP32 error is below the BF16 storage floor (l >= rank(A):
    # exact recovery up to the format) are compared by absolute difference.
    floor = 2.0 ** -8
    big = [(e, p) for e, p in zip(errs, plain_err) if p >= floor]
    ratio = max((e / p for e, p in big), default=None)
    absdiff = max(abs(e - p) for e, p in zip(errs, plain_err))
    worst = sorted(((e / p, i) for i, (e, p) in enumerate(zip(errs, plain_err)) if p >= floor),
                   reverse=True)[:3]
    worst = [dict(kind=reqs[i]["kind"], m=reqs[i]["m"], n=reqs[i]["n"], k=reqs[i]["k"],
                  q=reqs[i]["q"], err_served=errs[i], err_plain=plain_err[i], ratio=rt)
             for rt, i in worst]
    return {
        "metric": "CoR-UTV decompositions/s (roofline of the passes over A; p50/p99 latency)",
        "value": round(sat["decomps_per_s"], 3),
        "unit": "decomps/s",
        "n_gpus": 1, "steps": len(reqs), "warmup": 2,
        "ms_per_step": round(1e3 / sat["decomps_per_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": args.workload + ": " + w["desc"], "requests": len(reqs)},
        "served_saturation": sat,
        "served_poisson_0.8": dict(open_loop, arrival_rate_per_s=lam),
        "plain_fp32": {"decomps_per_s": plain_rate,
                       "p50_ms": float(np.percentile(plain_lat, 50)),
                       "p99_ms": float(np.percentile(plain_lat, 99))},
        "served_over_plain": sat["decomps_per_s"] / plain_rate,
        "accuracy": {"max_err_l_served_over_plain": ratio, "worst_requests": worst,
                     "requests_compared": len(big), "max_abs_err_l_difference": absdiff,
                     "bf16_floor": floor},
        "roofline": None,
        "cpu_baseline": None,
    }


def timed_plan(cu, torch, np, A, k, p, q, seed, args, colscale=None, profile_steps=20,
               opts=None, profile_kind=1, tune=False):
    """Plan one decomposition of the device matrix A, capture it into a HIP
    graph, replay `warmup` untimed and `steps` timed decompositions, then time
    the passes over A of eager runs of the same plan with HIP events on the
    plan's stream.  Returns the outputs and the timings."""
    dev = A.device
    m, n = A.shape
    l = k + p
    U = torch.empty((m, l), dtype=torch.float64, device=dev)
    T = torch.empty((l, l), dtype=torch.float64, device=dev)
    V = torch.empty((n, l), dtype=torch.float64, device=dev)
    perm = torch.empty((l,), dtype=torch.int32, device=dev)
    prob = cu.make_problem(A, k, p, q, seed=seed, U=U, T=T, V=V, perm=perm, colscale=colscale)
    splits = None
    if tune:  # the split tuner measures the passes' candidates on this matrix
        st, s_ax, s_atx = cu.cor_tune(prob, 3)
        cu.check(st, "cor_tune")
        splits = {"s_ax": s_ax, "s_atx": s_atx, "tuned": True}
    stream = torch.cuda.Stream()
    opts = opts if opts is not None else cu.cor_opts(0, 0)
    st, plan = cu.cor_plan_create([prob], opts)
    cu.check(st, "plan_create")
    graph = not args.no_graph
    try:
        with torch.cuda.stream(stream):
            if graph:
                cu.check(cu.cor_plan_capture(plan, stream), "plan_capture")
            for _ in range(args.warmup):
                cu.check(cu.cor_plan_run(plan, stream), "plan_run")
            stream.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev[0].record(stream)
            for i in range(args.steps):
                cu.check(cu.cor_plan_run(plan, stream), "plan_run")
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            # Pass timing: eager runs of a second plan over the same problem,
            # each pass launch bracketed by events on the plan's stream.
            st2, plan2 = cu.cor_plan_create([prob], opts)
            cu.check(st2, "plan_create")
            cu.cor_profile_enable(profile_kind)
            cu.cor_profile_read()
            for _ in range(profile_steps):
                cu.check(cu.cor_plan_run(plan2, stream), "plan_run")
            torch.cuda.synchronize()
            prof = cu.cor_profile_read()
            cu.cor_profile_enable(False)
            cu.cor_plan_destroy(plan2)
            # the result of the timed replays is in U, T, V (same plan, same outputs)
            cu.check(cu.cor_plan_run(plan, stream), "plan_run")
            st, info = cu.cor_plan_info(plan, 1, stream)
            cu.check(st, "plan_info")
    finally:
        cu.cor_plan_destroy(plan)
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    return dict(U=U, T=T, V=V, perm=perm, elapsed=t1 - t0, step_ms=step_ms, prof=prof,
                graph=graph, flags=info[0].flags, splits=splits)


def accuracy(torch, a64, U, T, V, k):
    """Explicit FP64 residuals of a result against the FP64 matrix, and the
    orthogonality of its factors."""
    l = T.shape[0]
    nA = torch.linalg.norm(a64)
    W = T @ V.T
    err_l = float(torch.linalg.norm(a64 - U @ W) / nA)
    err_k = float(torch.linalg.norm(a64 - U[:, :k] @ W[:k]) / nA)
    eye = torch.eye(l, device=U.device, dtype=torch.float64)
    return dict(err_l=err_l, err_k=err_k, orth_u=float(torch.linalg.norm(U.T @ U - eye)),
                orth_v=float(torch.linalg.norm(V.T @ V - eye)))


def pass_roofline(prec, l, prof, kernel="k_sketch (passes over A)", flops_per_elem=2):
    """Roofline of the passes over A (the dominant kernel): achieved
    algorithmic flops or bytes per launch over the mean launch time."""
    launches = max(1, prof["launches"])
    avg_s = prof["ms"] / launches / 1e3
    flops = prof["flops"] / launches
    nbytes = prof["bytes"] / launches
    # A pass does 2 l flops per element of A (the fused step 4 l): MFMA-bound
    # above the ridge (FP64 l >= 39, FP32 l >= 40 for a pass), HBM-bound below
    # it and in BF16/FP8.
    lr = l * flops_per_elem / 2
    if prec == "f64" and lr >= 39:
        bound, peak, unit = "mfma", PEAKS["f64"], "TFLOP/s"
        achieved = flops / avg_s / 1e12
    elif prec == "f32" and lr >= 40:
        bound, peak, unit = "mfma", PEAKS["f32"], "TFLOP/s"
        achieved = flops / avg_s / 1e12
    else:
        bound, peak, unit = "hbm", PEAKS["hbm_GBs"], "GB/s"
        achieved = nbytes / avg_s / 1e9
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "kernel": kernel,
            "avg_launch_us": round(avg_s * 1e6, 2), "launches_timed": prof["launches"],
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes}


def traffic_of(name, splits=None):
    """Calibrated HBM bytes per launch of the dominant kernel from the
    committed counters, if they were taken on the current source of that
    kernel (k_sketch.hip unless the file names another) and the same split
    counts."""
    tpath = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tr = json.load(f)
        same = splits is None or (tr.get("s_ax"), tr.get("s_atx")) == (splits["s_ax"],
                                                                         splits["s_atx"])
        src = tr.get("source", "k_sketch.hip")
        if tr.get("source_hash") == source_hash(src) and same:
            return tr.get("bytes_per_launch")
    return None


def cpu_threads():
    """BLAS threads for the numpy steps of the oracle's robust PCA (its
    CoR-UTV is single-threaded C): the host's cores this process may use, at
    most 16 (the host share of one GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def blas_limit(nthreads):
    """Context that pins numpy's BLAS pool to nthreads (the oracle's only
    multithreaded part)."""
    from threadpoolctl import threadpool_limits

    return threadpool_limits(limits=nthreads, user_api="blas")


def cpu_baseline_oracle(a64, k, p, q, seed, budget_rows=(300, 600)):
    """The FP64 oracle itself, end to end (Omega, 2q+2 products and QRs, the
    explicit compression pass, QRCP, U, V), on two leading row blocks of A
    with the full column count; its time is linear in the row count
    (t = a + b m: the n-side QRs and the l x l core do not depend on m), so
    the two runs give the time of the whole m-row decomposition."""
    import numpy as np

    import oracle

    m, n = a64.shape
    l = k + p
    om = oracle.omega(seed, n, l)
    times = []
    for r in budget_rows:  # the oracle's CoR-UTV is single-threaded C
        blk = np.ascontiguousarray(a64[:r].cpu().numpy())
        t = time.perf_counter()
        oracle.cor_utv(blk, k, p, q, om)
        times.append(time.perf_counter() - t)
    (r1, r2), (t1, t2) = budget_rows, times
    b = (t2 - t1) / (r2 - r1)
    a = t1 - b * r1
    est = a + b * m
    return dict(value=1.0 / est, unit="decomps/s", cores=1, kind="oracle",
                sample=f"oracle cor_utv end to end on the first {r1} and {r2} of {m} rows "
                       f"(n = {n}, k = {k}, p = {p}, q = {q}): {t1:.1f} s and {t2:.1f} s, "
                       f"linear in the rows -> {est:.1f} s per full decomposition",
                seconds_sampled=round(t1 + t2, 2))


C3_RULE = {  # at fixed error: the rule each pass format is held to
    "f64": "|eps - eps_oracle| <= 1e-12",
    "f32": "|eps - eps_oracle| <= 1e-5",
    "bf16": "eps <= 1.05 eps_oracle",
    "fp8": "eps <= 1.05 eps_oracle (not met: E4M3 noise above sigma_l); "
           "eps within 5 % of the stored-format oracle",
}


def bench_c3(args, w, cu, torch, np):
    """The 20000 x 10000 workload in every pass format: FP64 (the paper's
    arithmetic; the line's value), FP32, BF16 and FP8 with column scales.
    Each result is checked against the oracle's stored result for the same
    matrix and test matrix."""
    dev = torch.device("cuda:0")
    with open(os.path.join(ROOT, "tests", "golden", "c3_oracle.json")) as f:
        gold = json.load(f)
    gq = {}
    for fmt in ("bf16", "fp8"):
        pth = os.path.join(ROOT, "tests", "golden", f"c3_oracle_{fmt}.json")
        if os.path.exists(pth):
            with open(pth) as f:
                gq[fmt] = json.load(f)
    import inputs as I

    if args.input_cache and os.path.exists(args.input_cache):
        # a matrix saved by an earlier run of this workload (no QR on the device,
        # which matters under counter profilers)
        a64 = torch.from_numpy(np.load(args.input_cache, allow_pickle=False)).to(dev)
    else:
        a64, _ = I.config_matrix("c3", backend="torch", device=dev)
        if args.input_cache:
            np.save(args.input_cache, a64.cpu().numpy())
    k, p, q = gold["k"], gold["p"], gold["q"]
    l = k + p
    seed = gold["omega_seed"]
    # split tuning: from --tune-cache when it has this shape, else measured
    # here (and written to --tune-cache)
    loaded = {}
    if args.tune_cache and os.path.exists(args.tune_cache):
        cu.check(cu.cor_tune_load(args.tune_cache), "cor_tune_load")
        with open(args.tune_cache) as f:
            loaded = {(e["m"], e["n"], e["l"], e["prec"]): e for e in json.load(f)["entries"]}
    modes = {}
    for fmt in args.formats.split(","):
        colscale = None
        A32 = a64.float().contiguous()
        if fmt == "f64":
            A = a64
        elif fmt == "f32":
            A = A32
        elif fmt == "bf16":
            A = torch.empty(A32.shape, dtype=torch.bfloat16, device=dev)
            cu.check(cu.cor_quantize(A32, cu.COR_BF16, A), "quantize")
        else:
            A = torch.empty(A32.shape, dtype=torch.uint8, device=dev)
            colscale = torch.empty(A32.shape[1], dtype=torch.float32, device=dev)
            cu.check(cu.cor_quantize(A32, cu.COR_FP8, A, colscale), "quantize")
        if fmt != "f32":
            del A32
        torch.cuda.synchronize()
        ent = loaded.get((A.shape[0], A.shape[1], l, cu.PREC[fmt]))
        r = timed_plan(cu, torch, np, A, k, p, q, seed, args, colscale=colscale,
                       tune=not args.no_tune and ent is None)
        if ent is not None:
            r["splits"] = {"s_ax": ent["s_ax"], "s_atx": ent["s_atx"], "tuned": True,
                           "from": "tune cache"}
        del A
        acc = accuracy(torch, a64, r["U"], r["T"], r["V"], k)
        ratio = acc["err_l"] / gold["err_l"]
        if fmt == "f64":
            ok = abs(acc["err_l"] - gold["err_l"]) <= 1e-12 and \
                abs(acc["err_k"] - gold["err_k"]) <= 1e-12
        elif fmt == "f32":
            ok = abs(acc["err_l"] - gold["err_l"]) <= 1e-5
        elif fmt == "bf16":
            ok = ratio <= 1.05
        else:
            ok = ratio <= 1.05
        res = {
            "decomps_per_s": round(args.steps / r["elapsed"], 3),
            "ms_per_decomp": round(r["elapsed"] / args.steps * 1e3, 4),
            "latency_ms": {"p50": round(float(np.percentile(r["step_ms"], 50)), 4),
                           "p99": round(float(np.percentile(r["step_ms"], 99)), 4)},
            "err_l": acc["err_l"], "err_k": acc["err_k"],
            "err_l_over_oracle": ratio, "err_k_over_oracle": acc["err_k"] / gold["err_k"],
            "abs_diff_err_l": abs(acc["err_l"] - gold["err_l"]),
            "orth_u": acc["orth_u"], "orth_v": acc["orth_v"],
            "rule": C3_RULE[fmt], "at_fixed_error": bool(ok),
            "pass_roofline": pass_roofline(fmt, l, r["prof"]),
            "splits": r["splits"],
        }
        if fmt in gq:
            res["err_l_over_stored_format_oracle"] = acc["err_l"] / gq[fmt]["err_l"]
            if fmt == "fp8":
                res["stored_format_within_5pct"] = bool(
                    abs(acc["err_l"] / gq[fmt]["err_l"] - 1.0) <= 0.05)
        modes[fmt] = res
        head = fmt if fmt == args.formats.split(",")[0] else None
        if head:
            first = (fmt, r)
        print(f"# c3 {fmt}: {res['decomps_per_s']:.1f} decomps/s, eps/eps_oracle {ratio:.5f}, "
              f"pass {res['pass_roofline']['frac']:.3f} of {res['pass_roofline']['bound']} peak",
              file=sys.stderr, flush=True)
    if args.tune_cache and not os.path.exists(args.tune_cache):
        cu.check(cu.cor_tune_save(args.tune_cache), "cor_tune_save")
    fmt0, r0 = first
    main_mode = modes[fmt0]
    roofline = dict(main_mode["pass_roofline"])
    roofline["traffic"] = traffic_of(f"c3{fmt0}", r0["splits"])
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_oracle(a64, k, p, q, seed)
        cpu["cores_available"] = os.cpu_count()
    return {
        "metric": "CoR-UTV decompositions/s (roofline of the passes over A; p50/p99 latency) "
                  "at fixed error",
        "value": main_mode["decomps_per_s"],
        "unit": "decomps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_mode["ms_per_decomp"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": fmt0, "data": "synthetic",
        "config": {"workload": f"c3 {fmt0.upper()}: " + w["desc"], "m": a64.shape[0],
                   "n": a64.shape[1], "k": k, "l": l, "q": q, "graph": r0["graph"],
                   "splits": r0["splits"],
                   "omega_seed": seed},
        "latency_ms": main_mode["latency_ms"],
        "accuracy": {"err_l": main_mode["err_l"], "err_l_oracle": gold["err_l"],
                     "err_l_opt": gold["err_l_opt"], "err_k": main_mode["err_k"],
                     "err_k_oracle": gold["err_k"], "orth_u": main_mode["orth_u"],
                     "orth_v": main_mode["orth_v"], "rule": main_mode["rule"],
                     "at_fixed_error": main_mode["at_fixed_error"]},
        "roofline": roofline,
        "modes": modes,
        "cpu_baseline": cpu,
    }


def bench_tall(args, w, cu, torch, np):
    """Decompositions/s of a tall FP32 matrix with a small rank, where the
    passes are bound by HBM bandwidth: the fused power step (A^T (A X) in one
    read of A) against the two-pass step, same matrix and test matrix."""
    import inputs as I

    m, n, k, p, q, seed = w["m"], w["n"], w["k"], w["p"], w["q"], w["seed"]
    l = k + p
    low, sp = I.rpca_matrix(m, n, w["rank"], w["frac"], seed=seed)
    a64h = low + sp
    del low, sp
    a64 = torch.from_numpy(a64h).to("cuda:0")
    A = a64.float().contiguous()
    fused = timed_plan(cu, torch, np, A, k, p, q, 12345, args,
                       opts=cu.cor_opts(0, 0, 0, 0, 1), profile_kind=2)
    two = timed_plan(cu, torch, np, A, k, p, q, 12345, args, profile_kind=1)
    acc_f = accuracy(torch, a64, fused["U"], fused["T"], fused["V"], k)
    acc_2 = accuracy(torch, a64, two["U"], two["T"], two["V"], k)
    roof = pass_roofline("f32", l, fused["prof"], kernel="k_ata (fused power step)",
                         flops_per_elem=4)
    roof["traffic"] = traffic_of("tall")
    roof2 = pass_roofline("f32", l, two["prof"])
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_oracle(a64, k, p, q, 12345, budget_rows=(8000, 16000))
        cpu["cores_available"] = os.cpu_count()
    v_f = args.steps / fused["elapsed"]
    v_2 = args.steps / two["elapsed"]
    return {
        "metric": "CoR-UTV decompositions/s, fused power step (roofline of the fused pass)",
        "value": round(v_f, 3),
        "unit": "decomps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(fused["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tall: " + w["desc"], "m": m, "n": n, "k": k, "l": l, "q": q,
                   "graph": fused["graph"]},
        "latency_ms": {"p50": round(float(np.percentile(fused["step_ms"], 50)), 4),
                       "p99": round(float(np.percentile(fused["step_ms"], 99)), 4)},
        "two_pass": {"decomps_per_s": round(v_2, 3),
                     "ms_per_decomp": round(two["elapsed"] / args.steps * 1e3, 4),
                     "pass_roofline": roof2, "accuracy": acc_2},
        "speedup_over_two_pass": round(v_f / v_2, 3),
        "accuracy": dict(acc_f, err_l_minus_two_pass=acc_f["err_l"] - acc_2["err_l"],
                         rule="|eps_fused - eps_two_pass| <= 1e-5 (FP32)",
                         at_fixed_error=bool(abs(acc_f["err_l"] - acc_2["err_l"]) <= 1e-5)),
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def bench_host(args, w, cu, torch, np):
    """Decompositions/s with A in pinned host memory: every pass streams A
    over the host link in row panels, the copy of the next panel overlapping
    the kernels of the current one.  The bound is the host-to-device copy
    rate, calibrated here with a plain pinned copy of the same size."""
    import inputs as I

    m, n, k, p, q, seed = w["m"], w["n"], w["k"], w["p"], w["q"], w["seed"]
    l = k + p
    low, sp = I.rpca_matrix(m, n, w["rank"], w["frac"], seed=seed)
    a64h = low + sp
    del low, sp
    Ah = torch.from_numpy(a64h.astype(np.float32)).pin_memory()
    dev = torch.device("cuda:0")
    nbytes = m * n * 4
    # link calibration: the same bytes in one pinned host-to-device copy
    dst = torch.empty((m, n), dtype=torch.float32, device=dev)
    for _ in range(2):
        dst.copy_(Ah, non_blocking=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        dst.copy_(Ah, non_blocking=True)
    torch.cuda.synchronize()
    link = 3 * nbytes / (time.perf_counter() - t) / 1e9
    U = torch.empty((m, l), dtype=torch.float64, device=dev)
    T = torch.empty((l, l), dtype=torch.float64, device=dev)
    V = torch.empty((n, l), dtype=torch.float64, device=dev)
    pr = cu.make_problem(Ah, k, p, q, 12345, U, T, V)
    res = {}
    for name, fused in (("fused", 1), ("two_pass", 0)):
        opts = cu.cor_opts(0, 0, 0, 0, fused)
        for _ in range(max(1, args.warmup)):
            cu.check(cu.cor_utv_host(pr, opts, w["panel_rows"])[0], "cor_utv_host")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = []
        for _ in range(args.steps):
            ts = time.perf_counter()
            st, info = cu.cor_utv_host(pr, opts, w["panel_rows"])
            cu.check(st, "cor_utv_host")
            ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        passes = (q + 2) if fused else (2 * q + 2)
        acc = accuracy(torch, torch.from_numpy(a64h).to(dev), U, T, V, k) if name == "fused" \
            else None
        res[name] = dict(decomps_per_s=args.steps / el, ms=el / args.steps * 1e3,
                         p50=float(np.percentile(ms, 50)), p99=float(np.percentile(ms, 99)),
                         link_GBs=passes * nbytes / (el / args.steps) / 1e9, passes=passes,
                         accuracy=acc)
    f, tp = res["fused"], res["two_pass"]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_oracle(torch.from_numpy(a64h), k, p, q, 12345,
                                  budget_rows=(20000, 40000))
        cpu["cores_available"] = os.cpu_count()
    return {
        "metric": "CoR-UTV decompositions/s with A in host memory (host link rate against a "
                  "pinned copy)",
        "value": round(f["decomps_per_s"], 3),
        "unit": "decomps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(f["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "host: " + w["desc"], "m": m, "n": n, "k": k, "l": l, "q": q,
                   "panel_rows": w["panel_rows"]},
        "latency_ms": {"p50": round(f["p50"], 3), "p99": round(f["p99"], 3)},
        "link": {"bound": "host-to-device copy", "achieved_GBs": round(f["link_GBs"], 2),
                 "pinned_copy_GBs": round(link, 2), "frac": round(f["link_GBs"] / link, 4),
                 "streams_of_A": f["passes"]},
        "two_pass": {"decomps_per_s": round(tp["decomps_per_s"], 3), "ms": round(tp["ms"], 3),
                     "link_GBs": round(tp["link_GBs"], 2), "streams_of_A": tp["passes"],
                     "frac": round(tp["link_GBs"] / link, 4)},
        "speedup_over_two_pass": round(f["decomps_per_s"] / tp["decomps_per_s"], 3),
        "accuracy": f["accuracy"],
        "roofline": None,
        "cpu_baseline": cpu,
    }


def bench_rpca(args, w, cu, torch, np):
    """Robust PCA solves/s: each step is one whole ALM-CoRUTV solve (to
    zeta < 1e-5) of the same M, from the input in HBM to L and S in HBM."""
    import inputs as I
    import oracle

    n, rk, k, p, q, seed = w["n"], w["rank"], w["k"], w["p"], w["q"], w["seed"]
    low, sp = I.rpca_matrix(n, n, rk, w["frac"], seed=seed)
    M = torch.from_numpy(low + sp).to("cuda:0")
    lowd = torch.from_numpy(low).to("cuda:0")
    spd = torch.from_numpy(sp).to("cuda:0")
    stream = torch.cuda.Stream()
    infos, step_ms = [], []
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            L, S, info = cu.rpca(M, k, p, q, seed=seed, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            L, S, info = cu.rpca(M, k, p, q, seed=seed, stream=stream)
            step_ms.append((time.perf_counter() - ts) * 1e3)
            infos.append(info.as_dict())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # pass timing over one more solve, every pass launch bracketed by events
        cu.cor_profile_enable(True)
        cu.cor_profile_read()
        cu.rpca(M, k, p, q, seed=seed, stream=stream)
        torch.cuda.synchronize()
        prof = cu.cor_profile_read()
        cu.cor_profile_enable(False)
    lerr = float(torch.linalg.norm(L - lowd) / torch.linalg.norm(lowd))
    serr = float(torch.linalg.norm(S - spd) / torch.linalg.norm(spd))
    last = infos[-1]
    ok = last["rank"] == rk and last["zeta"] < 1e-5 and lerr < 1e-4 and serr < 1e-4
    roofline = pass_roofline("f64", k + p, prof)
    roofline["traffic"] = traffic_of("rpca")
    cpu = None
    if not args.no_cpu:
        # the oracle's ALM-CoRUTV on the same M for its first iterations; every
        # iteration does the same work (one CoR-UTV, the product, the updates),
        # so per-iteration time x the GPU solve's iteration count is the solve
        mh = low + sp
        nthr = cpu_threads()
        with blas_limit(nthr):
            t = time.perf_counter()
            oracle.rpca_alm(mh, k, p, q, omega_seed=seed, max_iter=w["cpu_iters"])
            dt = time.perf_counter() - t
        est = dt / w["cpu_iters"] * last["iters"]
        cpu = dict(value=1.0 / est, unit="solves/s", cores=nthr, kind="oracle",
                   sample=f"oracle rpca_alm on the same {n}x{n} M, first {w['cpu_iters']} "
                          f"iterations: {dt:.1f} s -> {est:.1f} s for the solve's "
                          f"{last['iters']} iterations",
                   seconds_sampled=round(dt, 2), cores_available=os.cpu_count())
    return {
        "metric": "ALM-CoRUTV robust PCA solves/s (to zeta < 1e-5)",
        "value": round(args.steps / (t1 - t0), 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rpca: " + w["desc"], "n": n, "rank": rk, "k": k, "l": k + p,
                   "q": q},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                       "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "result": {"iters": last["iters"], "rank": last["rank"], "zeta": last["zeta"],
                   "L_err": lerr, "S_err": serr, "recovered": ok},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--formats", default="f64,f32,bf16,fp8",
                    help="c3: pass formats to run, the first one is the line's value")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--input-cache", default="", metavar="NPY",
                    help="c3: load the 20000x10000 matrix from this .npy file if it exists, "
                         "else build it and save it there")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-cache", metavar="JSON",
                    default=os.path.join(ROOT, "paper_1810_07323_amd", "tune_mi355x.json"),
                    help="c3: split table to load (shapes it holds are not tuned again; "
                         "default: the table measured on MI355X for this workload); written "
                         "after the run when it does not exist")
    ap.add_argument("--no-tune", action="store_true",
                    help="c3: keep the rule's split counts instead of running the split tuner "
                         "on the matrix before timing")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "HBM byte counters against a kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X: multi-GPU runs are not part of this build "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_07323_amd as cu

    if args.copy_calib:
        nbytes = args.copy_calib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": nbytes, "copy_calib_bytes_written": nbytes,
                          "launches": 5}))
        return

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c3":
        print(json.dumps(bench_c3(args, w, cu, torch, np)))
        return
    if args.workload == "c4batched":
        print(json.dumps(bench_batched(args, w, cu, torch, np)))
        return
    if args.workload == "host":
        print(json.dumps(bench_host(args, w, cu, torch, np)))
        return
    if args.workload == "tall":
        print(json.dumps(bench_tall(args, w, cu, torch, np)))
        return
    if args.workload == "rpca":
        print(json.dumps(bench_rpca(args, w, cu, torch, np)))
        return
    if args.workload == "c5served":
        print(json.dumps(bench_served(args, w, cu, torch, np)))
        return
    k, p, q = w["k"], w["p"], w["q"]
    l = k + p
    m, n = w["m"], w["n"]
    a64, sig = make_input(w, dev)
    dtype = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[w["prec"]]
    A = a64.to(dtype).contiguous()
    r = timed_plan(cu, torch, np, A, k, p, q, 12345, args)
    acc = accuracy(torch, a64, r["U"], r["T"], r["V"], k)
    s2 = np.concatenate([sig ** 2, np.zeros(max(0, min(m, n) - len(sig)))])
    acc["err_l_opt"] = float(np.sqrt(s2[l:].sum() / s2.sum()))
    acc["err_k_opt"] = float(np.sqrt(s2[k:].sum() / s2.sum()))
    roofline = pass_roofline(w["prec"], l, r["prof"])
    roofline["traffic"] = traffic_of(args.workload)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_oracle(a64, k, p, q, 12345)
        cpu["cores_available"] = os.cpu_count()
    out = {
        "metric": "CoR-UTV decompositions/s (roofline of the passes over A; p50/p99 latency)",
        "value": round(args.steps / r["elapsed"], 3),
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["prec"],
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + w["desc"], "m": m, "n": n, "k": k, "l": l,
                   "q": q, "graph": r["graph"]},
        "latency_ms": {"p50": round(float(np.percentile(r["step_ms"], 50)), 4),
                       "p99": round(float(np.percentile(r["step_ms"], 99)), 4)},
        "accuracy": acc,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
