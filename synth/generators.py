"""Seeded input generators (host NumPy).  No part of PowerLU's arithmetic
lives here: only the construction of test matrices with prescribed singular
values, Gaussian test matrices and request streams."""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def spectrum(kind: str, count: int, **kw) -> np.ndarray:
    """Singular values sigma_1..sigma_count (1-based index i).

    kind: 'type1'  i^-2                      (Sec. 6.2, Matrix Type 1)
          'type2'  exp(-i/7)                 (Type 2)
          'type3'  1e-4 + 1/(1+exp(i-30))    (Type 3)
          'pow'    i^-alpha                  (alpha=kw['alpha'])
          'exp'    exp(-i/tau)               (tau=kw['tau'])
    """
    i = np.arange(1, count + 1, dtype=np.float64)
    if kind == "type1":
        return i ** -2.0
    if kind == "type2":
        return np.exp(-i / 7.0)
    if kind == "type3":
        # 1/(1+exp(i-30)) written to avoid overflow for large i
        return 1e-4 + np.exp(-np.logaddexp(0.0, i - 30.0))
    if kind == "pow":
        return i ** -float(kw["alpha"])
    if kind == "exp":
        return np.exp(-i / float(kw["tau"]))
    raise ValueError(kind)


def orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Q factor of a seeded rows x cols Gaussian matrix (orthonormal columns)."""
    G = rng.standard_normal((rows, cols))
    Q, R = np.linalg.qr(G, mode="reduced")
    # fix signs so the draw is a deterministic function of the seed
    return Q * np.sign(np.diag(R))[None, :]


def paper_type(t: int, n: int, seed: int, m: int | None = None,
               rank: int | None = None) -> np.ndarray:
    """Square (or m x n) matrix of Matrix Type t (Sec. 6.2) in float64.
    ``rank`` limits the construction to the leading singular triplets (the
    discarded tail is then exactly zero)."""
    m = n if m is None else m
    r = min(m, n) if rank is None else rank
    rng_u = np.random.default_rng(seed * 1000 + 0)
    rng_v = np.random.default_rng(seed * 1000 + 1)
    U = orthonormal(rng_u, m, r)
    V = orthonormal(rng_v, n, r)
    s = spectrum(f"type{t}", r)
    return (U * s[None, :]) @ V.T


def paper_type_family(n: int, seed: int, types=(1, 2, 3), dtype=np.float32,
                      chunk: int = 2000) -> dict:
    """Matrices of several Matrix Types (Sec. 6.2) at size n x n sharing one
    pair of random orthonormal factors U, V (the same draws ``paper_type``
    makes for ``seed``), so the two n x n QRs are paid once for all types:
    {t: U diag(sigma_t) V^T}, formed in float64 row chunks and rounded to
    ``dtype``."""
    U = orthonormal(np.random.default_rng(seed * 1000 + 0), n, n)
    V = orthonormal(np.random.default_rng(seed * 1000 + 1), n, n)
    out = {}
    for t in types:
        s = spectrum(f"type{t}", n)
        A = np.empty((n, n), dtype=dtype)
        for r0 in range(0, n, chunk):
            r1 = min(n, r0 + chunk)
            A[r0:r1] = (U[r0:r1] * s[None, :]) @ V.T
        out[t] = A
    return out


def lowrank_factors(m: int, n: int, sigma: np.ndarray, seed_left: int,
                    seed_right: int):
    """(X, sigma, Y) with X (m x r), Y (n x r) Q factors of seeded Gaussians."""
    r = len(sigma)
    X = orthonormal(np.random.default_rng(seed_left), m, r)
    Y = orthonormal(np.random.default_rng(seed_right), n, r)
    return X, np.asarray(sigma, np.float64), Y


def lowrank_plus_noise(m: int, n: int, sigma: np.ndarray, seed_left: int,
                       seed_right: int, noise: float = 0.0, seed_noise: int = 0,
                       dtype=np.float32, chunk: int = 2048) -> np.ndarray:
    """A = X diag(sigma) Y^T + noise * N(0,1), formed in float64 row chunks and
    rounded to ``dtype``.  The noise is drawn chunk by chunk from one seeded
    stream, so the result depends on the seeds only."""
    X, s, Y = lowrank_factors(m, n, sigma, seed_left, seed_right)
    A = np.empty((m, n), dtype=dtype)
    XS = X * s[None, :]
    rng = np.random.default_rng(seed_noise)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        blk = XS[r0:r1] @ Y.T
        if noise != 0.0:
            blk += noise * rng.standard_normal((r1 - r0, n))
        A[r0:r1] = blk
    return A


def gaussian_omega(rows: int, cols: int, seed: int, dtype=np.float32) -> np.ndarray:
    """N(0,1) test matrix (Sec. 1; Alg. 7)."""
    return np.random.default_rng(seed).standard_normal((rows, cols)).astype(dtype)


# ----------------------------------------------------------------------------
# Measurement workloads.
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    rank: int              # rank of the signal part
    sigma_kind: str
    sigma_kw: tuple
    noise: float           # per-entry noise scale
    params: tuple          # algorithm parameters as (key, value) pairs
    index: int             # seed base = 1000 * index

    def sigma(self) -> np.ndarray:
        return spectrum(self.sigma_kind, self.rank, **dict(self.sigma_kw))

    def param(self, key, default=None):
        return dict(self.params).get(key, default)


WORKLOADS = {
    # square 2000, Type 1 spectrum over the full rank, FP64 oracle in seconds
    "square2000_type1": Workload("square2000_type1", 2000, 2000, 2000, "type1", (),
                                 0.0, (("k", 20), ("p_over", 10), ("v", 3)), 1),
    # square 20000 rank 500 exp(-i/40) plus 1e-4 N(0,1)/sqrt(n) noise
    "square20000_exp40": Workload("square20000_exp40", 20000, 20000, 500, "exp",
                                  (("tau", 40.0),), 1e-4 / math.sqrt(20000),
                                  (("k", 100), ("p_over", 10), ("v", (2, 3, 4, 5))), 2),
    # square 32768 rank 1000 i^-1.5
    "square32768_pow15": Workload("square32768_pow15", 32768, 32768, 1000, "pow",
                                  (("alpha", 1.5),), 0.0,
                                  (("k", 200), ("p_over", 20), ("v", 4)), 3),
    # 30000 x 20000 rank 2000 exp(-i/50), fixed precision
    "rect30000x20000_exp50": Workload("rect30000x20000_exp50", 30000, 20000, 2000, "exp",
                                      (("tau", 50.0),), 0.0,
                                      (("eps", 1e-3), ("b", 32), ("l", 1600), ("v", 4)), 4),
}


def workload_matrix_factors(w: Workload, m: int | None = None, n: int | None = None):
    """Left/right factors and singular values of workload ``w`` (optionally
    at a reduced size m x n with the same spectrum and seeds)."""
    m = w.m if m is None else m
    n = w.n if n is None else n
    r = min(w.rank, m, n)
    s = w.sigma()[:r]
    return lowrank_factors(m, n, s, 1000 * w.index + 0, 1000 * w.index + 1)


def workload_matrix(w: Workload, m: int | None = None, n: int | None = None,
                    dtype=np.float32) -> np.ndarray:
    m = w.m if m is None else m
    n = w.n if n is None else n
    r = min(w.rank, m, n)
    noise = w.noise if (m, n) == (w.m, w.n) else (w.noise * math.sqrt(w.n / n) if w.noise else 0.0)
    return lowrank_plus_noise(m, n, w.sigma()[:r], 1000 * w.index + 0,
                              1000 * w.index + 1, noise, 1000 * w.index + 2, dtype)


def workload_slice(w: Workload, rows: int, cols: int, dtype=np.float32) -> np.ndarray:
    """The leading rows x cols block of workload ``w``'s matrix (signal part),
    formed directly from the full-size factors in float64 and rounded:
    X[:rows] diag(sigma) Y[:cols]^T.  Noise-free workloads only."""
    if w.noise:
        raise ValueError("workload_slice is for noise-free workloads")
    X, s, Y = workload_matrix_factors(w)
    return ((X[:rows] * s[None, :]) @ Y[:cols].T).astype(dtype)


# ----------------------------------------------------------------------------
# Request stream for the batched / serving form.
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    m: int
    n: int
    r: int
    mode: int           # 0 fixed rank, 1 fixed precision
    k: int
    p_over: int
    v: int
    eps: float
    b: int
    seed: int

    def sigma(self) -> np.ndarray:
        return spectrum("exp", self.r, tau=self.r / 4.0)

    def matrix(self, dtype=np.float32) -> np.ndarray:
        """Rank-r signal with singular values exp(-i/(r/4)) plus Gaussian noise
        scaled so that ||noise||_F = 1e-4 ||signal||_F."""
        s = self.sigma()
        sig_f = float(np.sqrt(np.sum(s * s)))
        noise = 1e-4 * sig_f / math.sqrt(self.m * self.n)
        return lowrank_plus_noise(self.m, self.n, s, self.seed * 10 + 0,
                                  self.seed * 10 + 1, noise, self.seed * 10 + 2, dtype)


def request_stream(count: int = 1024, rate_per_s: float = 200.0, seed: int = 5000,
                   mn_range=(512, 8192), r_range=(16, 256)) -> list:
    """Poisson arrivals (exponential gaps); m, n uniform in mn_range; r uniform
    in r_range; even ids fixed rank (k = r/2, p_over = 10, v uniform in 2..5),
    odd ids fixed precision (eps = 1e-3, b = 16, v = 4)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        m = int(rng.integers(mn_range[0], mn_range[1] + 1))
        n = int(rng.integers(mn_range[0], mn_range[1] + 1))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        v = int(rng.integers(2, 6))
        if i % 2 == 0:
            out.append(Request(i, t, m, n, r, 0, max(1, r // 2), 10, v, 0.0, 0, seed + 1 + i))
        else:
            out.append(Request(i, t, m, n, r, 1, 0, 0, 4, 1e-3, 16, seed + 1 + i))
    return out


def crafted_tie_matrix(m: int, c: int, seed: int) -> np.ndarray:
    """An m x c matrix (float64 values exactly representable in float32) on
    which partial pivoting meets exact ties at its steps while every
    elimination step stays exact in float32: the rows are C D with D a c x c
    upper triangular matrix (diagonal +-2, +-4 or +-8, integers in [-2, 2]
    above), C holding the unit rows, for each j one or two rows +-e_j plus
    +-1/4 e_t (t > j) -- these tie with row j of D in column j -- and filler
    rows with entries in {0, +-1/4, +-1/2}; rows shuffled.  Whether a given
    seed keeps every step exact (no filler row grows into a pivot) is a
    property checked by the tests that use it."""
    rng = np.random.default_rng(seed)
    D = np.triu(rng.integers(-2, 3, size=(c, c)).astype(np.float64), 1)
    D[np.arange(c), np.arange(c)] = np.exp2(rng.integers(1, 4, size=c)) * rng.choice([-1, 1], size=c)
    rows = [np.eye(c)]
    for j in range(c):
        for _ in range(rng.integers(1, 3)):
            r = np.zeros(c)
            r[j] = rng.choice([-1.0, 1.0])
            if j + 1 < c:
                r[rng.integers(j + 1, c)] += 0.25 * rng.choice([-1.0, 1.0])
            rows.append(r[None])
    nf = m - sum(x.shape[0] for x in rows)
    if nf < 0:
        raise ValueError("m too small for the tie rows")
    rows.append(rng.choice([0.0, 0.0, 0.25, -0.25, 0.5, -0.5], size=(nf, c)))
    X = np.concatenate(rows) @ D
    return X[rng.permutation(m)]


def sprand_csr(m: int, n: int, density: float, seed: int):
    """A sparse m x n matrix like MATLAB's ``sprand(m, n, density)`` (the
    sparse inputs of Sec. 6.1): uniform (0, 1) values at about
    density * m * n distinct positions drawn uniformly.  Returns compressed
    rows (indptr int64 m + 1, indices int32 ascending within each row, data
    float32)."""
    rng = np.random.default_rng(seed)
    target = int(round(density * m * n))
    # draw a few extra positions, drop repeats, keep the first target of them
    draw = rng.integers(0, m * n, size=int(target * 1.01) + 16, dtype=np.int64)
    _, first = np.unique(draw, return_index=True)
    lin = np.sort(draw[np.sort(first)][:target])
    rows = lin // n
    cols = (lin % n).astype(np.int32)
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=indptr[1:])
    data = rng.random(lin.size).astype(np.float32)
    return indptr, cols, data


def csr_dense(m: int, n: int, indptr, indices, data, dtype=np.float64) -> np.ndarray:
    """The dense matrix of compressed rows (repeated entries summed)."""
    A = np.zeros((m, n), dtype=dtype)
    rows = np.repeat(np.arange(m), np.diff(indptr))
    np.add.at(A, (rows, indices), data.astype(dtype))
    return A
