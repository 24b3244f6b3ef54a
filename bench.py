"""Throughput of the CoR-UTV hot path on one MI355X.

Default workload (the FP32 decomposition of the benchmark table):
A = 8000 x 8000, U, V random orthonormal 8000 x 500, sigma_i = exp(-i/40)
(i <= 500), stored FP32; k = 100, p = 10 (l = 110), q = 2.  One step is one
whole decomposition (Omega, 2q+2 passes over A with CholeskyQR2 after each,
M = R2^T, QRCP, U and V), replayed from a captured HIP graph of the plan.

Prints one JSON line: decompositions/s, p50/p99 step latency, the roofline of
the dominant kernel (the passes over A: FP32 MFMA-bound at l = 110) from HIP
events recorded around every pass launch inside the timed region, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
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
    "c2": dict(m=8000, n=8000, rank=500, spectrum="exp40", k=100, p=10, q=2, prec="f32", seed=202,
               desc="8000x8000 FP32, rank-500 Haar factors, sigma_i=exp(-i/40); k=100, l=110, q=2"),
    "c3bf16": dict(m=20000, n=10000, rank=10000, spectrum="pow15", k=200, p=20, q=2, prec="bf16",
                   seed=303, desc="20000x10000 BF16, sigma_i=i^-1.5; k=200, l=220, q=2"),
    "c1": dict(m=1000, n=1000, rank=1000, spectrum="c1", k=10, p=5, q=1, prec="f64", seed=101,
               noise=1e-6, desc="1000x1000 FP64, sigma 1 (i<=10) then 1e-3*0.9^(i-10); k=10, l=15, q=1"),
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


def source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1810_07323_amd", "csrc", "k_sketch.hip"), "rb") as f:
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


def cpu_baseline(a_host, w, budget_s=20.0):
    """Time the FP64 oracle on a row sample of A and scale to one decomposition.

    The oracle's cost is 2q+3 products with A or A^T (q+1 each way plus the
    explicit M = Q1^T (A Q2)), 2q+2 Householder QRs and the l x l core.  The
    sample runs the oracle's A X and A^T Y products over the first R rows of A
    (R chosen to keep the sample near `budget_s`) and one Householder QR of an
    m x l matrix; the products scale linearly in the rows.
    """
    import numpy as np

    import oracle

    m, n = a_host.shape
    l = w["k"] + w["p"]
    q = w["q"]
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n, l))
    # calibrate on a small block
    r0 = max(8, min(m, 64))
    t = time.perf_counter()
    oracle.gemm_nn(a_host[:r0], x)
    t_small = time.perf_counter() - t
    per_row_ax = t_small / r0
    rows = int(max(r0, min(m, (budget_s * 0.4) / max(per_row_ax, 1e-9))))
    blk = np.ascontiguousarray(a_host[:rows])
    t = time.perf_counter()
    oracle.gemm_nn(blk, x)
    t_ax = (time.perf_counter() - t) * m / rows
    y = rng.standard_normal((rows, l))
    t = time.perf_counter()
    oracle.gemm_tn(blk, y)
    t_atx = (time.perf_counter() - t) * m / rows
    t = time.perf_counter()
    oracle.qr(rng.standard_normal((m, l)))
    t_qr = time.perf_counter() - t
    total = (q + 1) * (t_ax + t_atx) + t_ax + (2 * q + 2) * t_qr
    return dict(value=1.0 / total, unit="decomps/s", cores=1, kind="oracle",
                sample=f"oracle A*X and A^T*Y over {rows} of {m} rows plus one {m}x{l} "
                       f"Householder QR, scaled to 2q+3={2 * q + 3} products and 2q+2 QRs "
                       f"(est. {total:.1f} s per decomposition)")


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
    # plain path: FP32, one request after another (warm the code paths first)
    for r in reqs[:2]:
        st, _ = cu.cor_utv_ex(cu.make_problem(mat(r), r["k"], r["p"], r["q"], r["seed"],
                                              *outputs(r)), opts)
        cu.check(st, "plain warmup")
    torch.cuda.synchronize()
    plain_err, plain_lat = [], []
    t0 = time.perf_counter()
    for r in reqs:
        ts = time.perf_counter()
        st, info = cu.cor_utv_ex(cu.make_problem(mat(r), r["k"], r["p"], r["q"], r["seed"],
                                                 *outputs(r)), opts)
        cu.check(st, "plain")
        plain_lat.append((time.perf_counter() - ts) * 1e3)
        plain_err.append(info.err_l)
    torch.cuda.synchronize()
    plain_rate = len(reqs) / (time.perf_counter() - t0)

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
        "accuracy": {"max_err_l_served_over_plain": ratio, "requests_compared": len(big),
                     "max_abs_err_l_difference": absdiff, "bf16_floor": floor},
        "roofline": None,
        "cpu_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
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
    if args.workload == "c4batched":
        print(json.dumps(bench_batched(args, w, cu, torch, np)))
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
    if w["prec"] != "f64":
        a_keep = a64
    else:
        a_keep = a64
    U = torch.empty((m, l), dtype=torch.float64, device=dev)
    T = torch.empty((l, l), dtype=torch.float64, device=dev)
    V = torch.empty((n, l), dtype=torch.float64, device=dev)
    perm = torch.empty((l,), dtype=torch.int32, device=dev)
    prob = cu.make_problem(A, k, p, q, seed=12345, U=U, T=T, V=V, perm=perm)
    stream = torch.cuda.Stream()
    st, plan = cu.cor_plan_create([prob], cu.cor_opts(0, 0))
    cu.check(st, "plan_create")
    graph = not args.no_graph
    with torch.cuda.stream(stream):
        if graph:
            cu.check(cu.cor_plan_capture(plan, stream), "plan_capture")
        for _ in range(args.warmup):
            cu.check(cu.cor_plan_run(plan, stream), "plan_run")
        stream.synchronize()
        # Timed region: K steps, events around every step (latency) and, in
        # eager mode, around every pass over A (roofline).
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        cu.cor_profile_enable(True)
        cu.cor_profile_read()  # reset counters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(args.steps):
            cu.check(cu.cor_plan_run(plan, stream), "plan_run")
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof_timed = cu.cor_profile_read()
        # Kernel timing of the passes over A: in graph mode the passes run
        # inside the graph, so a second, eager pass over the same steps
        # brackets each pass launch with events on the plan's stream.
        if graph:
            st2, plan2 = cu.cor_plan_create([prob], cu.cor_opts(0, 0))
            cu.check(st2, "plan_create")
            cu.cor_profile_read()
            for _ in range(min(args.steps, 20)):
                cu.check(cu.cor_plan_run(plan2, stream), "plan_run")
            torch.cuda.synchronize()
            prof = cu.cor_profile_read()
            cu.cor_plan_destroy(plan2)
        else:
            prof = prof_timed
        cu.cor_profile_enable(False)
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    elapsed = t1 - t0
    value = args.steps / elapsed

    # Accuracy of the timed result (fixed-error check): explicit FP64 residual
    # against the FP64 matrix, the optimum from the known spectrum, orthogonality.
    torch.cuda.synchronize()
    nA = torch.linalg.norm(a_keep)
    R = a_keep - (U @ T) @ V.T
    err_l = float(torch.linalg.norm(R) / nA)
    Rk = a_keep - (U[:, :k] @ T[:k, :]) @ V.T
    err_k = float(torch.linalg.norm(Rk) / nA)
    del R, Rk
    orth_u = float(torch.linalg.norm(U.T @ U - torch.eye(l, device=dev, dtype=torch.float64)))
    orth_v = float(torch.linalg.norm(V.T @ V - torch.eye(l, device=dev, dtype=torch.float64)))
    s2 = np.concatenate([sig ** 2, np.zeros(max(0, min(m, n) - len(sig)))])
    opt_l = float(np.sqrt(s2[l:].sum() / s2.sum()))
    opt_k = float(np.sqrt(s2[k:].sum() / s2.sum()))

    launches = max(1, prof["launches"])
    avg_s = prof["ms"] / launches / 1e3
    prec = w["prec"]
    flops_per_launch = prof["flops"] / launches
    bytes_per_launch = prof["bytes"] / launches
    if prec == "f32" and l >= 40:
        bound, peak, unit_r = "mfma", PEAKS["f32"], "TFLOP/s"
        achieved = flops_per_launch / avg_s / 1e12
    elif prec == "f64" and l >= 39:
        bound, peak, unit_r = "mfma", PEAKS["f64"], "TFLOP/s"
        achieved = flops_per_launch / avg_s / 1e12
    else:
        bound, peak, unit_r = "hbm", PEAKS["hbm_GBs"], "GB/s"
        achieved = bytes_per_launch / avg_s / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tr = json.load(f)
        if tr.get("source_hash") == source_hash():
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit_r,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "k_sketch (passes over A)", "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_flops_per_launch": flops_per_launch,
                "algorithmic_bytes_per_launch": bytes_per_launch}

    cpu = None
    if not args.no_cpu:
        a_host = a_keep.cpu().numpy()
        cpu = cpu_baseline(a_host, w)
        cpu["cores_available"] = os.cpu_count()

    out = {
        "metric": "CoR-UTV decompositions/s (roofline of the passes over A; p50/p99 latency)",
        "value": round(value, 3),
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + w["desc"], "m": m, "n": n, "k": k, "l": l,
                   "q": q, "graph": graph},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4)},
        "accuracy": {"err_l": err_l, "err_l_opt": opt_l, "err_k": err_k, "err_k_opt": opt_k,
                     "orth_u": orth_u, "orth_v": orth_v},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    cu.cor_plan_destroy(plan)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
