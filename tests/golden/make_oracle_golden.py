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

Run:  python tests/golden/make_oracle_golden.py c3   (and c2)
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
    main(sys.argv[1] if len(sys.argv) > 1 else "c3")
