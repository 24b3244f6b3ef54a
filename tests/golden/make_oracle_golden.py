"""Write the FP64 oracle's result on a full-size workload (c2 or c3).

  c3: A = U diag(sigma) V^T, U (20000 x 10000) and V (10000 x 10000) random
      orthonormal (QR of seeded Gaussians, sign-fixed), sigma_i = i^-1.5;
      k = 200, p = 20 (l = 220), q = 2.
  c2: 8000 x 8000, U, V random orthonormal 8000 x 500, sigma_i = exp(-i/40);
      k = 100, p = 10 (l = 110), q = 2.
The Gaussian test matrix is the documented counter-based stream (seed 3031
for c3, 2021 for c2).  The oracle runs once on the host (single thread,
minutes) and its errors and a sample of its factors go to <name>_oracle.json
beside this script, so that GPU runs at the full size are checked against it
without re-running the oracle.

Only the oracle and the seeded input generators are called here.  The device
builds the same matrix from the same Gaussians (its QR and products differ
only by rounding); the fingerprint lets a run confirm that.

With a storage format (bf16 or fp8) the script instead runs the oracle's
stored-format form of the method (each pass reads A and its skinny operand in
that format, products exact) on A quantised by the oracle's own quantiser
(A -> binary32 -> bfloat16, or E4M3 with per-column scales), and records its
errors against the FP64 A (what a user of that format gets) and against the
dequantised matrix; <name>_oracle_<fmt>.json.

Run:  python tests/golden/make_oracle_golden.py c3 [bf16|fp8]   (and c2)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OMEGA_SEED = {"c3": 3031, "c2": 2021}
DESC = {
    "c3": "20000x10000, U, V random orthonormal (seeds 607, 608), sigma_i = i^-1.5; "
          "k=200, p=20, q=2",
    "c2": "8000x8000, U, V random orthonormal 8000x500 (seeds 405, 406), "
          "sigma_i = exp(-i/40) (i <= 500); k=100, p=10, q=2",
}


def sample_rows(count, second=True):
    rows = {0, count // 2 - 1, count - 1}
    if second:
        rows.add(1)
    return sorted(rows)


def fingerprint(a):
    """Entries and norms that identify the matrix up to rounding."""
    return {
        "fro": float(np.linalg.norm(a)),
        "row0_head": a[0, :6].tolist(),
        "last_row_tail": a[-1, -6:].tolist(),
        "col_sums_head": a[:, :4].sum(axis=0).tolist(),
    }


def main_fmt(name, fmt):
    c = inputs.CONFIGS[name]
    k, p, q = c["k"], c["p"], c["q"]
    l = k + p
    t0 = time.time()
    a, sig = inputs.config_matrix(name)
    t_gen = time.time() - t0
    m, n = a.shape
    a32 = a.astype(np.float32)
    t0 = time.time()
    if fmt == "bf16":
        h = oracle.quantize_bf16(a32)
        aq = oracle.bf16_to_f64(h)
        cs = None
        deq = aq
    else:
        codes, cs = oracle.quantize_fp8(a32)
        aq = oracle.fp8_to_f64(np.arange(256))[codes]
        deq = aq * cs.astype(np.float64)[None, :]
    del a32
    t_q = time.time() - t0
    print(f"matrix {a.shape} built in {t_gen:.1f} s, quantised in {t_q:.1f} s", flush=True)
    om = oracle.omega(OMEGA_SEED[name], n, l)
    t0 = time.time()
    r = oracle.cor_utv_fmt(aq, fmt, k, p, q, om, colscale=cs)
    t_orc = time.time() - t0
    print(f"stored-format oracle in {t_orc:.1f} s", flush=True)
    del aq
    t0 = time.time()
    met = oracle.metrics(a, r["U"], r["T"], r["V"], k)
    met_q = oracle.metrics(deq, r["U"], r["T"], r["V"], k)
    t_met = time.time() - t0
    print(f"metrics in {t_met:.1f} s: vs A {met}; vs deq(A) {met_q}", flush=True)
    nrm = float(np.linalg.norm(a))
    out = {
        "workload": DESC[name], "format": fmt,
        "m": m, "n": n, "k": k, "p": p, "q": q, "matrix_seed": c["seed"],
        "omega_seed": OMEGA_SEED[name],
        "err_l": met["err_l"], "err_k": met["err_k"],
        "err_l_vs_stored": met_q["err_l"], "err_k_vs_stored": met_q["err_k"],
        "orth_u": met["orth_u"], "orth_v": met["orth_v"],
        "format_error": float(np.linalg.norm(a - deq) / nrm),
        "T_diag": np.diag(r["T"]).tolist(),
        "fingerprint": fingerprint(a),
        "host_seconds": {"generate": t_gen, "quantise": t_q, "oracle": t_orc,
                         "metrics": t_met},
    }
    with open(os.path.join(HERE, f"{name}_oracle_{fmt}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("written", flush=True)


def main(name):
    c = inputs.CONFIGS[name]
    k, p, q = c["k"], c["p"], c["q"]
    l = k + p
    t0 = time.time()
    a, sig = inputs.config_matrix(name)
    t_gen = time.time() - t0
    print(f"matrix {a.shape} built in {t_gen:.1f} s", flush=True)
    m, n = a.shape
    om = oracle.omega(OMEGA_SEED[name], n, l)
    t0 = time.time()
    r = oracle.cor_utv(a, k, p, q, om, want_intermediates=True)
    t_orc = time.time() - t0
    print(f"oracle decomposition in {t_orc:.1f} s", flush=True)
    t0 = time.time()
    met = oracle.metrics(a, r["U"], r["T"], r["V"], k)
    t_met = time.time() - t0
    print(f"metrics in {t_met:.1f} s: {met}", flush=True)
    s2 = np.concatenate([np.asarray(sig, dtype=np.float64) ** 2, np.zeros(max(0, n - len(sig)))])
    out = {
        "workload": DESC[name],
        "m": m, "n": n, "k": k, "p": p, "q": q, "matrix_seed": c["seed"],
        "omega_seed": OMEGA_SEED[name],
        "err_l": met["err_l"], "err_k": met["err_k"],
        "orth_u": met["orth_u"], "orth_v": met["orth_v"],
        "err_l_opt": float(np.sqrt(s2[l:].sum() / s2.sum())),
        "err_k_opt": float(np.sqrt(s2[k:].sum() / s2.sum())),
        "m_minus_r2t": float(r["diag"][0]), "min_pivot_gap": float(r["diag"][1]),
        "perm": r["perm"].tolist(),
        "T_diag": np.diag(r["T"]).tolist(),
        "T_row0": r["T"][0, :].tolist(),
        "U_rows": {str(i): r["U"][i].tolist() for i in sample_rows(m)},
        "V_rows": {str(i): r["V"][i].tolist() for i in sample_rows(n, second=False)},
        "fingerprint": fingerprint(a),
        "host_seconds": {"generate": t_gen, "oracle": t_orc, "metrics": t_met},
    }
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("written", flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 2:
        main_fmt(sys.argv[1], sys.argv[2])
    else:
        main(sys.argv[1] if len(sys.argv) > 1 else "c3")
