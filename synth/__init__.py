"""Seeded synthetic inputs for the SpMV library, its oracle and its benchmark.

This module only draws random numbers and lays out the sparsity patterns the
workloads are made of.  It performs none of the sparse-matrix arithmetic that
is being tested (no products, no sums over rows, no format conversion beyond
emitting triplets in row-major order), so both the HIP path and the CPU oracle
can take their inputs from here without sharing any of the method.

Every matrix comes back as COO triplets ``(row, col, val)`` (int32, int32,
float64 unless stated) with rows ascending and columns ascending inside a row;
callers that test the COO->CSR conversion shuffle or duplicate them.

Workload recipes (the paper's Holstein-Hubbard matrix, its Section 4.2 test
case, is not available, so these synthetic patterns stand in for it):

* ``laplacian3d(m)``: 7-point Laplacian on an m^3 grid, lexicographic index
  i + m*j + m*m*k, 6 on the diagonal and -1 for each existing neighbour
  (Dirichlet boundary: missing neighbours are dropped).
* ``powerlaw``: nonsymmetric, row lengths from a truncated power law
  P(L) ~ L^-alpha on [1, 2000] with alpha = 1.6929 (mean 15.0); ceil(L/2)
  columns uniform in the band [i-1000, i+1000] clipped to [0, n), floor(L/2)
  uniform over [0, n); all distinct within a row; values N(0,1).
* ``sym_diagonals``: the diagonal plus 12 secondary diagonals at offsets drawn
  without replacement from [1, n/4], mirrored so the matrix is symmetric; the
  shape of the paper's Hamiltonian (a dozen heavy outer diagonals, symmetric).
* ``many_matrices``: independent square matrices, n log-uniform in
  [1e3, 2e5], row lengths uniform in {5..40}, columns uniform and distinct.
* ``banded_uniform``: 16 columns uniform in the band [i-5000, i+5000] and 4
  uniform over [0, n), distinct; N(0,1) values divided by the largest absolute
  row sum so that the infinity norm of the matrix is 1.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20091026
POWERLAW_ALPHA = 1.6929


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    """Generator for workload ``config`` (1..5); ``salt`` separates streams."""
    return np.random.default_rng([BASE_SEED + config, salt])


def uniform_vector(n: int, rng: np.random.Generator, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1], drawn in float64 and cast (round to nearest) to ``dtype``."""
    return rng.uniform(-1.0, 1.0, size=n).astype(dtype)


# ---------------------------------------------------------------------------
# helpers


def _row_ids(lengths: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)


def _sort_rowmajor(rows: np.ndarray, cols: np.ndarray, n_cols: int):
    key = rows.astype(np.int64) * np.int64(n_cols) + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    return order


def _dedupe(rng, rows, cols, kinds, n_cols, redraw):
    """Redraw entries until no (row, col) pair repeats.

    ``redraw(rows_subset, kinds_subset)`` returns fresh columns.  Only rows that
    still hold a repeat are re-examined, so the loop touches a shrinking set.
    """
    active = np.arange(len(rows), dtype=np.int64)
    while len(active):
        r = rows[active]
        c = cols[active]
        key = r.astype(np.int64) * np.int64(n_cols) + c.astype(np.int64)
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(len(ks), dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        bad = active[order[dup]]
        bad.sort()
        cols[bad] = redraw(rows[bad], kinds[bad])
        bad_rows = np.unique(rows[bad])
        active = np.flatnonzero(np.isin(rows, bad_rows))
    return cols


def _finish(rows, cols, vals, n_cols):
    order = _sort_rowmajor(rows, cols, n_cols)
    return (rows[order].astype(np.int32), cols[order].astype(np.int32), vals[order])


# ---------------------------------------------------------------------------
# workloads


def laplacian3d(m: int = 20):
    """7-point Laplacian on an m x m x m grid (index i + m*j + m*m*k)."""
    idx = np.arange(m ** 3, dtype=np.int64)
    i = idx % m
    j = (idx // m) % m
    k = idx // (m * m)
    rows, cols, vals = [], [], []
    # neighbours in ascending column order: -m^2, -m, -1, 0, +1, +m, +m^2
    for off, ok in ((-m * m, k > 0), (-m, j > 0), (-1, i > 0), (0, None),
                    (1, i < m - 1), (m, j < m - 1), (m * m, k < m - 1)):
        sel = idx if ok is None else idx[ok]
        rows.append(sel)
        cols.append(sel + off)
        vals.append(np.full(len(sel), 6.0 if off == 0 else -1.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return _finish(r, c, v, m ** 3) + (m ** 3, m ** 3)


def powerlaw_lengths(n: int, rng, lmax: int = 2000, alpha: float = POWERLAW_ALPHA):
    L = np.arange(1, lmax + 1, dtype=np.float64)
    p = L ** -alpha
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    u = rng.random(n)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.int64)


def powerlaw(n: int = 2_000_000, lmax: int = 2000, band: int = 1000,
             alpha: float = POWERLAW_ALPHA, seed_config: int = 2):
    """Power-law row lengths, half band / half uniform columns, N(0,1) values."""
    rng = rng_for(seed_config)
    lengths = powerlaw_lengths(n, rng, lmax, alpha)
    nb = (lengths + 1) // 2
    nu = lengths // 2
    rows_b = _row_ids(nb)
    rows_u = _row_ids(nu)
    lo = np.maximum(np.arange(n, dtype=np.int64) - band, 0)
    hi = np.minimum(np.arange(n, dtype=np.int64) + band, n - 1)
    width = hi - lo + 1
    # band columns: long rows draw without replacement row by row, short rows
    # draw with replacement and are fixed up by the shared dedupe pass.
    cols_b = np.empty(len(rows_b), dtype=np.int64)
    starts_b = np.concatenate(([0], np.cumsum(nb)))
    long_rows = np.flatnonzero(nb > 32)
    short_mask = np.repeat(nb <= 32, nb)
    rs = rows_b[short_mask]
    cols_b[short_mask] = lo[rs] + (rng.random(len(rs)) * width[rs]).astype(np.int64)
    for r in long_rows:
        s = starts_b[r]
        cols_b[s:s + nb[r]] = lo[r] + rng.choice(width[r], size=nb[r], replace=False)
    cols_u = rng.integers(0, n, size=len(rows_u), dtype=np.int64)
    rows = np.concatenate([rows_b, rows_u])
    cols = np.concatenate([cols_b, cols_u])
    kinds = np.concatenate([np.zeros(len(rows_b), np.int8), np.ones(len(rows_u), np.int8)])

    def redraw(rr, kk):
        out = rng.integers(0, n, size=len(rr), dtype=np.int64)
        bandsel = kk == 0
        rb = rr[bandsel]
        out[bandsel] = lo[rb] + (rng.random(len(rb)) * width[rb]).astype(np.int64)
        return out

    cols = _dedupe(rng, rows, cols, kinds, n, redraw)
    vals = rng.standard_normal(len(rows))
    return _finish(rows, cols, vals, n) + (n, n)


def sym_offsets(n: int, ndiag: int, rng) -> np.ndarray:
    return np.sort(rng.choice(np.arange(1, n // 4 + 1), size=ndiag, replace=False)).astype(np.int64)


def sym_diagonals(n: int = 6_000_000, ndiag: int = 12, seed_config: int = 3):
    """Diagonal plus ``ndiag`` mirrored secondary diagonals, N(0,1) values.

    Draw order: offsets, then the upper-triangle values of each offset in
    ascending offset order, then the diagonal.  Entry (i, i+d) and its mirror
    (i+d, i) hold the same value.
    """
    rng = rng_for(seed_config)
    offs = sym_offsets(n, ndiag, rng)
    upper = [rng.standard_normal(n - int(d)) for d in offs]
    diag = rng.standard_normal(n)
    i = np.arange(n, dtype=np.int64)
    # 2*ndiag+1 candidate slots per row in ascending column order
    slot_off = np.concatenate([-offs[::-1], [0], offs])
    cand = i[:, None] + slot_off[None, :]
    valid = (cand >= 0) & (cand < n)
    vals = np.zeros(cand.shape, dtype=np.float64)
    for t, d in enumerate(offs[::-1]):           # lower slots: (i, i-d) = U_d[i-d]
        sel = i >= d
        vals[sel, t] = upper[ndiag - 1 - t][i[sel] - d]
    vals[:, ndiag] = diag
    for t, d in enumerate(offs):                 # upper slots: (i, i+d) = U_d[i]
        sel = i + d < n
        vals[sel, ndiag + 1 + t] = upper[t][i[sel]]
    rows = np.broadcast_to(i[:, None], cand.shape)[valid]
    return (rows.astype(np.int32), cand[valid].astype(np.int32), vals[valid], n, n)


def heavy_diagonals_band(n: int = 6_000_000, npairs: int = 6, fill: float = 0.7, band: int = 500,
                         band_per_row: float = 2.3, seed_config: int = 6):
    """Symmetric pattern shaped like the paper's Hamiltonian: the diagonal,
    ``npairs`` mirrored pairs of outer secondary diagonals (offsets drawn
    without replacement from [2*band, n/4], each position filled with
    probability ``fill``) and entries scattered over the band |i - j| <= band
    (2 or 3 upper entries per row, mean ``band_per_row``, distinct, mirrored).
    N(0,1) values, mirrored pairs equal.  With the defaults 12.7 entries per
    row, 56% of them on the outer diagonals, 36% in the band.

    Draw order: offsets, the outer diagonals' fill masks and values in
    ascending offset order, the band offsets (redrawn on collision), the band
    values, the diagonal."""
    rng = rng_for(seed_config)
    offs = np.sort(rng.choice(np.arange(2 * band, n // 4 + 1), size=npairs, replace=False)).astype(np.int64)
    up_r, up_c, up_v = [], [], []
    for d in offs:
        i = np.arange(n - d, dtype=np.int64)
        keep = rng.random(len(i)) < fill
        up_r.append(i[keep])
        up_c.append(i[keep] + d)
        up_v.append(rng.standard_normal(int(keep.sum())))
    p3 = band_per_row - 2.0
    lengths = 2 + (rng.random(n) < p3).astype(np.int64)
    rows = _row_ids(lengths)
    kinds = np.zeros(len(rows), np.int8)

    def draw(rr, kk):
        return rr + rng.integers(1, band + 1, size=len(rr), dtype=np.int64)

    cols = draw(rows, kinds)
    cols = _dedupe(rng, rows, cols, kinds, n + band + 1, draw)
    inside = cols < n
    up_r.append(rows[inside])
    up_c.append(cols[inside])
    up_v.append(rng.standard_normal(int(inside.sum())))
    diag = rng.standard_normal(n)
    r = np.concatenate(up_r)
    c = np.concatenate(up_c)
    v = np.concatenate(up_v)
    i = np.arange(n, dtype=np.int64)
    rows_all = np.concatenate([r, c, i])
    cols_all = np.concatenate([c, r, i])
    vals_all = np.concatenate([v, v, diag])
    return _finish(rows_all, cols_all, vals_all, n) + (n, n)


def sym_diagonals_offsets(n: int = 6_000_000, ndiag: int = 12, seed_config: int = 3):
    return sym_offsets(n, ndiag, rng_for(seed_config))


def _uniform_distinct_rows(rng, n_rows, n_cols, lengths):
    rows = _row_ids(lengths)
    cols = rng.integers(0, n_cols, size=len(rows), dtype=np.int64)
    kinds = np.zeros(len(rows), np.int8)
    cols = _dedupe(rng, rows, cols, kinds, n_cols,
                   lambda rr, kk: rng.integers(0, n_cols, size=len(rr), dtype=np.int64))
    return rows, cols


def many_matrix_sizes(count: int = 512, nmin: int = 1000, nmax: int = 200_000,
                      seed_config: int = 4):
    rng = rng_for(seed_config, 1)
    return np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)


def many_matrices(count: int = 512, nmin: int = 1000, nmax: int = 200_000,
                  lmin: int = 5, lmax: int = 40, seed_config: int = 4):
    """Independent square matrices for the batched form (float32 values and x).

    Yields ``(row, col, val_f32, n, x_f32)`` per matrix, in order.
    """
    sizes = many_matrix_sizes(count, nmin, nmax, seed_config)
    for m, n in enumerate(sizes):
        rng = rng_for(seed_config, 100 + m)
        n = int(n)
        lengths = rng.integers(lmin, min(lmax, n) + 1, size=n).astype(np.int64)
        rows, cols = _uniform_distinct_rows(rng, n, n, lengths)
        vals = rng.standard_normal(len(rows)).astype(np.float32)
        r, c, v = _finish(rows, cols, vals, n)
        x = uniform_vector(n, rng, np.float32)
        yield r, c, v, n, x


def banded_uniform(n: int = 4_000_000, nband: int = 16, band: int = 5000, nunif: int = 4,
                   seed_config: int = 5, dtype=np.float32):
    """Rows of nband band columns plus nunif uniform ones, scaled to norm_inf = 1."""
    rng = rng_for(seed_config)
    L = nband + nunif
    lengths = np.full(n, L, dtype=np.int64)
    rows = _row_ids(lengths)
    kinds = np.tile(np.concatenate([np.zeros(nband, np.int8), np.ones(nunif, np.int8)]), n)
    lo = np.maximum(np.arange(n, dtype=np.int64) - band, 0)
    hi = np.minimum(np.arange(n, dtype=np.int64) + band, n - 1)
    width = hi - lo + 1

    def draw(rr, kk):
        out = rng.integers(0, n, size=len(rr), dtype=np.int64)
        b = kk == 0
        rb = rr[b]
        out[b] = lo[rb] + (rng.random(len(rb)) * width[rb]).astype(np.int64)
        return out

    cols = draw(rows, kinds)
    cols = _dedupe(rng, rows, cols, kinds, n, draw)
    vals = rng.standard_normal(len(rows))
    r, c, v = _finish(rows, cols, vals, n)
    rowsum = np.bincount(r, weights=np.abs(v), minlength=n)
    v = (v / rowsum.max()).astype(dtype)
    return r, c, v, n, n


# ---------------------------------------------------------------------------
# small patterns for tests


def random_pattern(n_rows: int, n_cols: int, density: float, rng, *,
                   integer: bool = False, lo: int = -8, hi: int = 8,
                   empty_rows: float = 0.0, long_rows: int = 0, long_len: int = 0):
    """Random sparse pattern with optional empty rows and a few long rows.

    Values are N(0,1), or integers in [lo, hi] (never 0) when ``integer``.
    """
    lengths = rng.binomial(n_cols, density, size=n_rows).astype(np.int64)
    if empty_rows > 0:
        lengths[rng.random(n_rows) < empty_rows] = 0
    if long_rows:
        pick = rng.choice(n_rows, size=min(long_rows, n_rows), replace=False)
        lengths[pick] = min(long_len, n_cols)
    rows = _row_ids(lengths)
    cols = np.empty(len(rows), dtype=np.int64)
    starts = np.concatenate(([0], np.cumsum(lengths)))
    for r in np.flatnonzero(lengths):
        cols[starts[r]:starts[r + 1]] = rng.choice(n_cols, size=lengths[r], replace=False)
    if integer:
        mag = rng.integers(1, max(abs(lo), abs(hi)) + 1, size=len(rows))
        sign = np.where(rng.random(len(rows)) < 0.5, -1, 1)
        vals = np.clip(sign * mag, lo, hi).astype(np.float64)
        vals[vals == 0] = 1.0
    else:
        vals = rng.standard_normal(len(rows))
    return _finish(rows, cols, vals, n_cols) + (n_rows, n_cols)


def random_symmetric(n: int, density: float, rng, *, integer: bool = False,
                     empty_rows: float = 0.0, long_rows: int = 0, long_len: int = 0):
    """Random symmetric pattern: a random_pattern whose entries on or above the
    diagonal are kept and mirrored below it (the mirror holds the same value).
    Rows are in ascending column order."""
    r, c, v, _, _ = random_pattern(n, n, density, rng, integer=integer, empty_rows=empty_rows,
                                   long_rows=long_rows, long_len=long_len)
    up = c >= r
    r, c, v = r[up].astype(np.int64), c[up].astype(np.int64), v[up]
    off = c > r
    rows = np.concatenate([r, c[off]])
    cols = np.concatenate([c, r[off]])
    vals = np.concatenate([v, v[off]])
    return _finish(rows, cols, vals, n) + (n, n)


def integer_vector(n: int, rng, lo: int = -8, hi: int = 8) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=n).astype(np.float64)


# ---------------------------------------------------------------------------
# index streams for the access-pattern microbenchmarks (Section 4.1, Table 1)


def index_stream(kind: str, n: int, k: float, rng, sd: float = 0.0) -> np.ndarray:
    """n int64 indices into the input vector.

    * ``"IS"``: constant stride, ind(i) = k*i (k integer).
    * ``"IR"``: random strides of mean k: every element of the vector is kept
      with probability p = 1/k, so the gaps between kept elements are
      geometric on {1, 2, ...} with mean k and variance k(k-1); the first
      kept element is the first success, at gap-1.
    * ``"GAUSS"``: strides round(N(k, sd^2)), started far enough from 0
      (six standard deviations of the walk) that backward jumps stay
      inside the vector; the rare walk that leaves [0, ...) is clipped.
    """
    if kind == "IS":
        return np.arange(n, dtype=np.int64) * int(k)
    if kind == "IR":
        return np.cumsum(rng.geometric(1.0 / k, size=n).astype(np.int64)) - 1
    if kind == "GAUSS":
        steps = np.rint(rng.normal(k, sd, size=n)).astype(np.int64)
        start = int(math.ceil(6.0 * sd * math.sqrt(n)))
        return np.maximum(start + np.cumsum(steps), 0)
    raise ValueError(kind)
