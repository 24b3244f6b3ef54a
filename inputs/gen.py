"""Seeded matrix and request generators (input construction only).

Every function takes an explicit integer seed.  Small inputs are built with
numpy (LAPACK QR for the orthonormal factors); large ones may be built with
torch on a device (``backend="torch"``), which is the only fast way to draw a
20000x10000 random orthonormal factor.  Results are float64.

Both backends draw the Gaussian matrices with numpy's seeded generator
(``gauss="numpy"``, the default), so the host and the device build the same
matrix up to the rounding of their QR and product routines: a value stored by
a host script for a large workload describes the matrix a device run builds.
``gauss="device"`` draws on the device instead (fast, for workloads of many
matrices that nothing stored refers to).
"""

from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Workload table.  Sizes follow the paper's problem statement (A is m x n,
# k <= l < min(m, n), l = k + p, q power steps) at the shapes of the
# benchmark workloads (1000^2 FP64, 8000^2 FP32, 20000x10000 BF16).
# ---------------------------------------------------------------------------
CONFIGS = {
    # 1000x1000 FP64, Haar U,V, sigma_i = 1 (i<=10), 1e-3*0.9^(i-10) after,
    # i.i.d. N(0, (1e-6)^2) noise; k=10, p=5, q in {0,1}.
    "c1": dict(m=1000, n=1000, k=10, p=5, q=(0, 1), prec="f64", spectrum="c1",
               rank=1000, noise=1e-6, seed=101),
    # 8000x8000, rank 500, sigma_i = exp(-i/40); k=100, l=110, q=2; FP32 passes.
    "c2": dict(m=8000, n=8000, k=100, p=10, q=2, prec="f32", spectrum="exp40",
               rank=500, noise=0.0, seed=202),
    # 20000x10000, sigma_i = i^-1.5 (full rank); k=200, l=220, q=2.
    "c3": dict(m=20000, n=10000, k=200, p=20, q=2, prec="bf16", spectrum="pow15",
               rank=10000, noise=0.0, seed=303),
}


def spectrum(kind: str, r: int, k: int | None = None) -> np.ndarray:
    """Singular values sigma_1..sigma_r (1-based index i) of a named spectrum."""
    i = np.arange(1, r + 1, dtype=np.float64)
    if kind == "c1":
        return np.where(i <= 10, 1.0, 1e-3 * 0.9 ** (i - 10))
    if kind == "exp40":
        return np.exp(-i / 40.0)
    if kind == "pow15":
        return i ** -1.5
    if kind == "expk":
        assert k is not None
        return np.exp(-i / float(k))
    raise ValueError(kind)


def gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) rows x cols from numpy's seeded generator (PCG64)."""
    return np.random.default_rng(seed).standard_normal((rows, cols))


def haar(rows: int, cols: int, seed: int, backend: str = "numpy", device=None,
         gauss: str = "numpy"):
    """Random orthonormal rows x cols factor: Q of QR(G), columns * sign(diag R).

    G is i.i.d. N(0,1).  With the sign correction Q is Haar distributed
    (Mezzadri, Notices AMS 2007), and unique given G.
    """
    if backend == "numpy":
        g = gaussian(rows, cols, seed)
        q, r = np.linalg.qr(g)
        s = np.sign(np.diag(r))
        s[s == 0] = 1.0
        return q * s
    import torch

    if gauss == "numpy":
        g = torch.from_numpy(gaussian(rows, cols, seed)).to(device)
    else:
        gen = torch.Generator(device=device).manual_seed(seed)
        g = torch.randn(rows, cols, generator=gen, dtype=torch.float64, device=device)
    q, r = torch.linalg.qr(g)
    del g
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s


def lowrank(m: int, n: int, sigma, seed: int, noise: float = 0.0,
            backend: str = "numpy", device=None, gauss: str = "numpy"):
    """A = U diag(sigma) V^T (+ noise * N(0,1)), U m x r, V n x r random orthonormal.

    Returns (A, sigma) with sigma as given (the exact singular values of the
    noiseless part).
    """
    r = len(sigma)
    if backend == "numpy":
        u = haar(m, r, seed * 2 + 1)
        v = haar(n, r, seed * 2 + 2)
        a = (u * np.asarray(sigma)[None, :]) @ v.T
        if noise:
            a = a + noise * gaussian(m, n, seed * 2 + 3)
        return a, np.asarray(sigma)
    import torch

    u = haar(m, r, seed * 2 + 1, backend="torch", device=device, gauss=gauss)
    v = haar(n, r, seed * 2 + 2, backend="torch", device=device, gauss=gauss)
    s = torch.as_tensor(np.asarray(sigma), dtype=torch.float64, device=device)
    a = (u * s[None, :]) @ v.T
    del u, v
    if noise:
        if gauss == "numpy":
            a += noise * torch.from_numpy(gaussian(m, n, seed * 2 + 3)).to(device)
        else:
            gen = torch.Generator(device=device).manual_seed(seed * 2 + 3)
            a += noise * torch.randn(m, n, generator=gen, dtype=torch.float64, device=device)
    return a, np.asarray(sigma)


def config_matrix(name: str, backend: str = "numpy", device=None, scale: float = 1.0):
    """The matrix of a named workload; ``scale`` < 1 shrinks m, n and the rank
    proportionally (parity tests run the same recipe at a size the oracle
    finishes in seconds)."""
    c = CONFIGS[name]
    m = max(8, int(round(c["m"] * scale)))
    n = max(8, int(round(c["n"] * scale)))
    r = min(m, n, max(1, int(round(c["rank"] * scale))))
    sig = spectrum(c["spectrum"], r)
    a, sig = lowrank(m, n, sig, c["seed"], noise=c["noise"], backend=backend, device=device)
    return a, sig


def noisy_lowrank(gap: float, seed: int, n: int = 1000, k: int = 20):
    """NoisyLowRank-I (gap=0.01) / -II (gap=0.1) of the singular-value study.

    sigma = linspace(1, 1e-9, n) with sigma_j = 0 for j > k, random orthonormal
    U, V; plus a Gaussian E rescaled to spectral norm gap * sigma_k.  The paper's
    phrase "decrease linearly from 1 to 1e-9" is read over all n values (the
    printed SVD curve of Fig. 1 has sigma_20 ~ 0.98, which rules out reaching
    1e-9 by j = 20).
    """
    sig = np.linspace(1.0, 1e-9, n)[:k]
    u = haar(n, k, seed * 2 + 1)
    v = haar(n, k, seed * 2 + 2)
    a1 = (u * sig[None, :]) @ v.T
    e = np.random.default_rng(seed * 2 + 3).standard_normal((n, n))
    e *= gap * sig[k - 1] / np.linalg.norm(e, 2)
    return a1 + e


def rpca_matrix(m: int, n: int, rank: int, frac: float, seed: int, mag: float = 80.0):
    """Robust-PCA input L + S: L = G1 G2^T (G1 m x r, G2 n x r, i.i.d. N(0,1));
    S has round(frac*m*n) positions drawn uniformly without replacement with
    values +-mag equiprobable (synthetic recovery experiment, Tables I/II)."""
    rng = np.random.default_rng(seed)
    g1 = rng.standard_normal((m, rank))
    g2 = rng.standard_normal((n, rank))
    low = g1 @ g2.T
    s = np.zeros(m * n)
    cnt = int(round(frac * m * n))
    pos = rng.choice(m * n, size=cnt, replace=False)
    s[pos] = mag * np.where(rng.random(cnt) < 0.5, -1.0, 1.0)
    return low, s.reshape(m, n)


def gaussian_omega(n: int, l: int, seed: int) -> np.ndarray:
    """An i.i.d. N(0,1) n x l test matrix, handed to both sides of a comparison."""
    return np.random.default_rng(10_000_019 + seed).standard_normal((n, l))


def batched_problems(count: int, seed: int, mn_lo=256, mn_hi=4096, k_lo=8, k_hi=64,
                     extra=8, q=1, rank_mult=39):
    """Problem list of the batched workload: m, n ~ U{mn_lo..mn_hi},
    k ~ U{k_lo..k_hi}, l = k + extra, sigma_i = exp(-i/k) for
    i <= min(m, n, rank_mult*k).  Returns dicts with the matrix seed; the matrix
    itself is built with ``lowrank`` on demand."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(mn_lo, mn_hi + 1))
        n = int(rng.integers(mn_lo, mn_hi + 1))
        k = int(rng.integers(k_lo, k_hi + 1))
        l = k + extra
        l = min(l, min(m, n) - 1)
        k = min(k, l)
        r = min(m, n, rank_mult * k)
        out.append(dict(m=m, n=n, k=k, p=l - k, q=q, rank=r, seed=seed * 1000 + i))
    return out


def served_requests(count: int, seed: int, rate: float, mn_lo=512, mn_hi=16384,
                    k_lo=16, k_hi=256, p=8, rpca_frac=0.1, pool=64):
    """Open-loop Poisson request list of the served workload.

    Arrival gaps ~ Exp(rate); m, n log-uniform in [mn_lo, mn_hi]; k ~ U{k_lo..k_hi};
    q ~ U{0,1,2}.  A fraction ``rpca_frac`` are robust-PCA shaped requests
    (76800 x 2000, rank 5 + 5% outliers of +-80).  Decaying-spectrum requests
    reference one of ``pool`` pre-built matrices by index so that a matrix can
    be reused across requests.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    shapes = []
    prng = np.random.default_rng(seed + 1)
    for j in range(pool):
        m = int(round(math.exp(prng.uniform(math.log(mn_lo), math.log(mn_hi)))))
        n = int(round(math.exp(prng.uniform(math.log(mn_lo), math.log(mn_hi)))))
        shapes.append((m, n))
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        q = int(rng.integers(0, 3))
        if rng.random() < rpca_frac:
            out.append(dict(t=t, kind="rpca", m=76800, n=2000, k=16, p=p, q=q,
                            seed=seed * 1000 + i))
        else:
            j = int(rng.integers(0, pool))
            m, n = shapes[j]
            k = int(rng.integers(k_lo, k_hi + 1))
            k = min(k, min(m, n) - p - 1)
            out.append(dict(t=t, kind="decay", pool=j, m=m, n=n, k=k, p=p, q=q,
                            seed=seed * 1000 + i))
    return out
