"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws numbers and builds matrices; it contains none of the
qdot arithmetic (no exponents, bins, scores, quantisation or sums), so the
oracle and the device path can both take their inputs from here without
sharing any of the method's code.

Every generator takes an explicit integer seed and uses numpy's PCG64.  The
value laws follow the workloads the qdot paper studies:

* ``log_uniform_pair``: components s * 10**u with u uniform on [lo, hi] and
  an equiprobable sign, x and y independent.  This is the law of the single
  qdot workloads (n = 1e5 and n = 2**27 at u in [-20, 20]).
* ``paper_dist_a`` / ``paper_dist_b``: the two synthetic families of the
  error-bound experiments (Sec. 4.1): s * 2**p with s ~ U[0.5, 1) and p
  uniform on [-t/2, t/2] (family A) or normal with standard deviation t/2
  (family B); p is rounded to an integer.  Both are positive.
* ``poisson2d_csr``: the 5-point Dirichlet Laplacian on an m x m grid
  (diagonal 4, neighbours -1), CSR with int32 indices.  It stands in for the
  HPCCG matrices the paper's CG study uses (Sec. 4.2), which are not
  available here.
* ``laplacian3d_csr``: the 7-point Dirichlet Laplacian on an m**3 grid
  (diagonal 6, neighbours -1), standing in for the paper's random graph
  Laplacians in the power-method study (Sec. 4.3).
* ``ragged_batch``: many independent qdot instances with log-uniform lengths
  in [1e2, 1e6] and tolerances drawn from {1e-4, 1e-6, 1e-8}.
* ``banded_pair``: x and y made of contiguous bands of random length, each
  band at its own magnitude level (normal values times 2**level), so that
  whole index ranges of products lie far below the largest ones: the banded
  precision pattern of a solver's vectors (Sec. 4.2), where tiles of the
  index order fall entirely into the perforated class.
* ``cancelling_pair``: products of random sign and size whose sum cancels to
  a chosen relative level (the last component is set from the exact sum of
  the others), so that the largest product exponent lies far above the
  exponent of the dot product (the case Thm 3.4 covers).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = [
    "rng",
    "log_uniform_pair",
    "paper_dist_a",
    "paper_dist_b",
    "normal_vector",
    "unit_vector",
    "poisson2d_csr",
    "laplacian3d_csr",
    "ragged_batch",
    "cg_grid_sides",
    "log_uniform_pair_torch",
    "cancelling_pair",
    "banded_pair",
    "paired_cancelling_torch",
    "paper_dist_torch",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _log_uniform(g: np.random.Generator, n: int, lo: float, hi: float,
                 out: np.ndarray) -> None:
    chunk = 1 << 22
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = g.uniform(lo, hi, e - s)
        sign = np.where(g.integers(0, 2, e - s) == 0, 1.0, -1.0)
        np.power(10.0, u, out=u)
        out[s:e] = sign * u


def log_uniform_pair(n: int, seed: int, lo: float = -20.0, hi: float = 20.0):
    """x, y in FP64, i.i.d. components +-10**U[lo, hi] (independent signs)."""
    g = rng(seed)
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    _log_uniform(g, n, lo, hi, x)
    _log_uniform(g, n, lo, hi, y)
    return x, y


def _paper_family(n: int, t: float, seed: int, normal: bool):
    g = rng(seed)
    out = []
    for _ in range(2):
        s = g.uniform(0.5, 1.0, n)
        if normal:
            p = np.rint(g.normal(0.0, 0.5 * t, n))
        else:
            p = np.rint(g.uniform(-0.5 * t, 0.5 * t, n))
        out.append(np.ldexp(s, p.astype(np.int64)))
    return out[0], out[1]


def paper_dist_a(n: int, t: float, seed: int):
    """Family A of the error-bound study: s * 2**p, p ~ U[-t/2, t/2]."""
    return _paper_family(n, t, seed, normal=False)


def paper_dist_b(n: int, t: float, seed: int):
    """Family B of the error-bound study: s * 2**p, p ~ N(0, t/2)."""
    return _paper_family(n, t, seed, normal=True)


def normal_vector(n: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(n)


def unit_vector(n: int, seed: int) -> np.ndarray:
    v = rng(seed).standard_normal(n)
    return v / np.sqrt(np.dot(v, v))


def _stencil_csr(shape, diag: float):
    """CSR of the Dirichlet Laplacian stencil on a tensor grid.

    Row order is lexicographic with the last axis fastest.  Within a row the
    column indices are ascending, so every consumer sums a row in the same
    order.
    """
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    cols = [idx]
    vals = [np.full(shape, diag)]
    for ax in range(len(shape)):
        for d in (-1, 1):
            nb = np.roll(idx, -d, axis=ax)
            valid = np.ones(shape, dtype=bool)
            sl = [slice(None)] * len(shape)
            sl[ax] = slice(-1, None) if d == 1 else slice(0, 1)
            valid[tuple(sl)] = False
            cols.append(np.where(valid, nb, -1))
            vals.append(np.where(valid, -1.0, 0.0))
    C = np.stack([c.reshape(n) for c in cols], axis=1)
    V = np.stack([v.reshape(n) for v in vals], axis=1)
    order = np.argsort(np.where(C < 0, np.iinfo(np.int64).max, C), axis=1,
                       kind="stable")
    C = np.take_along_axis(C, order, axis=1)
    V = np.take_along_axis(V, order, axis=1)
    keep = C >= 0
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    col = C[keep].astype(np.int32)
    val = V[keep].astype(np.float64)
    return rowptr.astype(np.int32), col, val


def poisson2d_csr(m: int):
    """5-point Laplacian, m x m grid, Dirichlet boundary: (rowptr, col, val)."""
    return _stencil_csr((m, m), 4.0)


def laplacian3d_csr(m: int):
    """7-point Laplacian, m x m x m grid, Dirichlet boundary."""
    return _stencil_csr((m, m, m), 6.0)


def random_spd_csr(n: int, extra_per_row: int, seed: int):
    """Random sparse symmetric strictly diagonally dominant matrix (SPD):
    each row gets about 2 * extra_per_row off-diagonal entries -U(0.1, 1)
    at random columns (symmetrised), and a diagonal of 1 + the absolute row
    sum.  Rows are sorted by column: (rowptr, col, val) as int32/int32/f64.
    Used for rows longer than the stencil matrices have."""
    g = rng(seed)
    i = np.repeat(np.arange(n, dtype=np.int64), extra_per_row)
    j = g.integers(0, n, n * extra_per_row)
    keep = i != j
    i, j = i[keep], j[keep]
    v = -g.uniform(0.1, 1.0, i.shape[0])
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    vals = np.concatenate([v, v])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, rows, cols, vals = key[order], rows[order], cols[order], vals[order]
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    grp = np.cumsum(first) - 1
    vals = np.bincount(grp, weights=vals)          # merge duplicate positions
    rows, cols = rows[first], cols[first]
    diag = 1.0 + np.bincount(rows, weights=np.abs(vals), minlength=n)
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def ragged_batch(count: int, seed: int, n_lo: float = 1e2, n_hi: float = 1e6,
                 tols=(1e-4, 1e-6, 1e-8), mag_lo: float = -20.0,
                 mag_hi: float = 20.0, max_total: int | None = None):
    """A ragged batch of qdot instances stored back to back.

    Returns (offsets[int64, count+1], x_cat, y_cat, tols[float64, count]).
    Instance j occupies [offsets[j], offsets[j+1]).  Lengths are
    round(10**U[log10 n_lo, log10 n_hi]); when ``max_total`` is given the
    lengths are scaled down so that their sum does not exceed it (used for
    small test batches).
    """
    g = rng(seed)
    lens = np.rint(10.0 ** g.uniform(np.log10(n_lo), np.log10(n_hi), count))
    lens = lens.astype(np.int64)
    if max_total is not None and lens.sum() > max_total:
        lens = np.maximum(1, (lens * (max_total / lens.sum())).astype(np.int64))
    offsets = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    tol = np.asarray(tols, dtype=np.float64)[g.integers(0, len(tols), count)]
    x = np.empty(total, dtype=np.float64)
    y = np.empty(total, dtype=np.float64)
    _log_uniform(g, total, mag_lo, mag_hi, x)
    _log_uniform(g, total, mag_lo, mag_hi, y)
    return offsets, x, y, tol


def cg_grid_sides(count: int, seed: int, lo_exp: float = 5.0,
                  hi_exp: float = 9.0) -> np.ndarray:
    """Grid sides m_j = round(2**U[lo_exp, hi_exp]) for a batch of 2D CG systems."""
    g = rng(seed)
    return np.rint(2.0 ** g.uniform(lo_exp, hi_exp, count)).astype(np.int64)


def log_uniform_pair_torch(n: int, seed: int, device="cuda:0"):
    """Same law as ``log_uniform_pair`` drawn on the device with a seeded
    torch generator (fast for n = 2**27; a different random stream from the
    numpy generator)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = []
    for _ in range(2):
        u = torch.rand(n, generator=g, dtype=torch.float64, device=device)
        u.mul_(40.0).sub_(20.0)
        v = torch.pow(10.0, u)
        del u
        s = torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int8)
        v.mul_(1.0 - 2.0 * s.to(torch.float64))
        del s
        out.append(v)
    return out[0], out[1]


def banded_pair(n: int, seed: int, levels=(0, -10, -25, -40, -70), mean_band: float = 3000.0):
    """x, y in FP64 of bands with geometric lengths (mean `mean_band`, not
    aligned to any tile) whose components are standard normal times
    2**level, the level drawn per band from `levels` (x and y share the
    band layout and the level)."""
    g = rng(seed)
    x = g.standard_normal(n)
    y = g.standard_normal(n)
    i = 0
    while i < n:
        length = int(g.geometric(1.0 / mean_band))
        lv = float(levels[int(g.integers(0, len(levels)))])
        x[i:i + length] *= 2.0 ** lv
        y[i:i + length] *= 2.0 ** lv
        i += length
    return x, y


def cancelling_pair(n: int, seed: int, rel: float):
    """x, y in FP64 with x.y about rel * |x_n y_n|: n - 1 products of
    normal sign and size 10**U[-3, 3], then x_n = -(their exact sum) *
    (1 + rel * U[-1, 1]) and y_n = 1 (the exact sum is taken in rationals
    and rounded once)."""
    g = rng(seed)
    x = g.standard_normal(n) * 10.0 ** g.uniform(-3.0, 3.0, n)
    y = g.standard_normal(n)
    d = float(sum((Fraction(a) * Fraction(b) for a, b in zip(x[:-1].tolist(), y[:-1].tolist())),
                  Fraction(0)))
    x[-1] = -d * (1.0 + rel * g.uniform(-1.0, 1.0))
    y[-1] = 1.0
    return x, y


def cancelling_wide_f32(n: int, seed: int, lo: float = -18.0, hi: float = 18.0,
                        rel: float = 1e-3):
    """x, y as float32 vectors whose products span 10**U[lo, hi] with random
    signs (y = 1), and whose sum cancels: the last x is set, in float32, to
    minus the exact sum of the others times (1 + rel * U[-1, 1]).  With the
    default range the products span more exponents than any FP32 number."""
    g = rng(seed)
    x = (g.choice([-1.0, 1.0], n) * 10.0 ** g.uniform(lo, hi, n)).astype(np.float32)
    y = np.ones(n, dtype=np.float32)
    d = float(sum((Fraction(float(a)) for a in x[:-1].tolist()), Fraction(0)))
    x[-1] = np.float32(-d * (1.0 + rel * g.uniform(-1.0, 1.0)))
    return x, y


def paired_cancelling_torch(n: int, seed: int, rel: float, device="cuda:0"):
    """x, y in FP64 on the device, n even: a = +-10**U[-3, 3], b normal,
    u = U[-1, 1] (m = n/2 each), x = [a, -a (1 + rel u)], y = [b, b].  The
    products of the two halves cancel pair by pair up to rel, so x.y is about
    rel * sqrt(m) times a typical product while e_max is that of the largest."""
    import torch

    assert n % 2 == 0
    m = n // 2
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    e = torch.rand(m, generator=g, dtype=torch.float64, device=device)
    e.mul_(6.0).sub_(3.0)
    a = torch.pow(10.0, e)
    del e
    s = torch.randint(0, 2, (m,), generator=g, device=device, dtype=torch.int8)
    a.mul_(1.0 - 2.0 * s.to(torch.float64))
    del s
    b = torch.randn(m, generator=g, dtype=torch.float64, device=device)
    u = torch.rand(m, generator=g, dtype=torch.float64, device=device)
    u.mul_(2.0 * rel).sub_(rel).add_(1.0)
    x = torch.cat([a, -(a * u)])
    del a, u
    y = torch.cat([b, b])
    return x, y


def paper_dist_torch(n: int, t: float, seed: int, family: str, device="cuda:0"):
    """Families A and B of the error-bound study drawn on the device (the
    law of ``paper_dist_a`` / ``paper_dist_b``, another random stream):
    s * 2**p with s ~ U[0.5, 1) and p = round(U[-t/2, t/2]) (family "A") or
    round(N(0, t/2)) (family "B"), x and y independent."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = []
    for _ in range(2):
        s = torch.rand(n, generator=g, dtype=torch.float64, device=device)
        s.mul_(0.5).add_(0.5)
        if family == "A":
            p = torch.rand(n, generator=g, dtype=torch.float64, device=device)
            p.mul_(t).sub_(0.5 * t)
        else:
            p = torch.randn(n, generator=g, dtype=torch.float64, device=device)
            p.mul_(0.5 * t)
        out.append(torch.ldexp(s, torch.round(p)))
        del s, p
    return out[0], out[1]
