"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: brute force on a dense copy,
exact integer arithmetic, a closed form, a library routine, or an identity the
paper states (Section 2: NUJDS with unroll = number of diagonals is CRS in the
permuted basis; RBJDS with block size 1 is row by row; plain JDS is the
block-size-n limit; JDS, NUJDS and NBJDS share one storage).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lap():
    r, c, v, n, _ = synth.laplacian3d(20)
    return oracle.csr_from_coo(n, n, r, c, v)


def rand_csr(seed, n_rows=40, n_cols=50, density=0.15, integer=False, empty=0.1, long_rows=0,
             long_len=0):
    rng = np.random.default_rng(seed)
    r, c, v, nr, nc = synth.random_pattern(n_rows, n_cols, density, rng, integer=integer,
                                           empty_rows=empty, long_rows=long_rows, long_len=long_len)
    return oracle.csr_from_coo(nr, nc, r, c, v), rng


def dense_of(A):
    M = np.zeros((A.n_rows, A.n_cols))
    rows = A.row_index()
    M[rows, A.col] = A.val
    return M


# --------------------------------------------------------------------------- CRS


@pytest.mark.parametrize("seed", range(6))
def test_crs_matches_dense_brute_force(seed):
    """Dense y_i = sum over ascending j of A[i,j]*x[j] (nonzeros only), in Python floats."""
    A, rng = rand_csr(seed, n_rows=int(10 + 9 * seed), n_cols=int(64 - 5 * seed))
    x = rng.uniform(-1, 1, A.n_cols)
    M = dense_of(A)
    want = np.zeros(A.n_rows)
    for i in range(A.n_rows):
        s = 0.0
        for j in range(A.n_cols):
            if M[i, j] != 0.0:
                s = s + float(M[i, j]) * float(x[j])
        want[i] = s
    got = oracle.spmv_crs(A, x)
    assert np.array_equal(got, want)
    # and numpy's dense product agrees to rounding
    D = oracle.row_absdot(A, x)
    assert oracle.rel_err(got, M @ x, D).max() <= 1e-14


def test_crs_alpha_beta():
    A, rng = rand_csr(11)
    x = rng.uniform(-1, 1, A.n_cols)
    y0 = rng.uniform(-1, 1, A.n_rows)
    M = dense_of(A)
    got = oracle.spmv_crs(A, x, y0, alpha=2.5, beta=-0.75)
    assert np.allclose(got, 2.5 * (M @ x) - 0.75 * y0, rtol=0, atol=1e-13)
    y_nan = np.full(A.n_rows, np.nan)
    got0 = oracle.spmv_crs(A, x, y_nan, alpha=1.0, beta=0.0)   # beta = 0 never reads y
    assert np.all(np.isfinite(got0))


@pytest.mark.parametrize("seed", range(4))
def test_crs_integer_exact(seed):
    """Small-integer values and x: every partial sum is an exact integer."""
    A, rng = rand_csr(100 + seed, n_rows=60, n_cols=70, density=0.3, integer=True, long_rows=2,
                      long_len=70)
    x = synth.integer_vector(A.n_cols, rng)
    got = oracle.spmv_crs(A, x)
    rows = A.row_index()
    want = [0] * A.n_rows
    for k in range(A.nnz):
        want[rows[k]] += int(A.val[k]) * int(x[A.col[k]])
    assert got.tolist() == [float(w) for w in want]


def test_crs_scipy_cross_check():
    A, rng = rand_csr(7, n_rows=500, n_cols=400, density=0.05)
    x = rng.uniform(-1, 1, A.n_cols)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    got = oracle.spmv_crs(A, x)
    assert oracle.rel_err(got, S @ x, oracle.row_absdot(A, x)).max() <= 1e-14


def test_spmm_columns_are_spmv():
    A, rng = rand_csr(8, n_rows=50, n_cols=45, density=0.2, integer=True)
    X = rng.integers(-8, 9, size=(A.n_cols, 5)).astype(np.float64)
    Y = oracle.spmm_crs(A, X)
    M = dense_of(A)
    assert np.array_equal(Y, M @ X)       # integers: exact either way


# --------------------------------------------------------------------------- Laplacian


def sine_mode(p, q, r, m=20):
    idx = np.arange(m ** 3)
    i, j, k = idx % m, (idx // m) % m, idx // (m * m)
    h = m + 1
    return (np.sin(p * np.pi * (i + 1) / h) * np.sin(q * np.pi * (j + 1) / h)
            * np.sin(r * np.pi * (k + 1) / h))


def test_laplacian_structure_golden():
    g = json.load(open(os.path.join(GOLD, "laplacian20.json")))
    A = lap()
    assert A.n_rows == g["n"] and A.nnz == g["nnz"]
    counts = np.bincount(A.row_lengths())
    assert {str(L): int(c) for L, c in enumerate(counts) if c} == g["row_length_counts"]
    J = oracle.jds_from_csr(A)
    assert J.jd_ptr.tolist() == g["jd_ptr"]


def test_laplacian_sine_modes():
    g = json.load(open(os.path.join(GOLD, "laplacian20.json")))
    A = lap()
    for e in g["eigen"]:
        p, q, r = e["mode"]
        lam = 6 - 2 * math.cos(p * math.pi / 21) - 2 * math.cos(q * math.pi / 21) - 2 * math.cos(r * math.pi / 21)
        assert abs(lam - e["lambda"]) <= 1e-13
        v = sine_mode(p, q, r)
        Av = oracle.spmv_crs(A, v)
        D = oracle.row_absdot(A, v)
        assert oracle.rel_err(Av, lam * v, D).max() <= 1e-12


# --------------------------------------------------------------------------- COO -> CRS


def test_csr_from_coo_duplicates_and_order():
    rng = np.random.default_rng(3)
    n_rows, n_cols = 30, 25
    k = 400
    row = rng.integers(0, n_rows, k).astype(np.int32)
    col = rng.integers(0, n_cols, k).astype(np.int32)   # many duplicates
    val = rng.standard_normal(k)
    val[::17] = 0.0                                      # explicit zeros stay
    A = oracle.csr_from_coo(n_rows, n_cols, row, col, val)
    # brute force: dense accumulation in input order, Python floats
    acc = {}
    for t in range(k):
        key = (int(row[t]), int(col[t]))
        acc[key] = acc[key] + float(val[t]) if key in acc else float(val[t])
    keys = sorted(acc)
    assert A.nnz == len(keys)
    assert list(zip(A.row_index().tolist(), A.col.tolist())) == keys
    assert A.val.tolist() == [acc[kk] for kk in keys]
    # scipy agrees on the pattern and (to rounding) on the sums
    S = sp.coo_matrix((val, (row, col)), shape=(n_rows, n_cols)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    assert np.array_equal(S.indptr, A.row_ptr)
    assert np.array_equal(S.indices, A.col)
    assert np.allclose(S.data, A.val, rtol=0, atol=1e-14)


def test_csr_from_coo_rejects_bad_index():
    with pytest.raises(ValueError):
        oracle.csr_from_coo(3, 3, np.array([0, 3], np.int32), np.array([0, 0], np.int32), np.ones(2))
    with pytest.raises(ValueError):
        oracle.csr_from_coo(3, 3, np.array([0, 1], np.int32), np.array([0, -1], np.int32), np.ones(2))


def test_csr_from_coo_empty():
    A = oracle.csr_from_coo(4, 5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert A.nnz == 0 and A.row_ptr.tolist() == [0] * 5
    assert oracle.spmv_crs(A, np.ones(5)).tolist() == [0.0] * 4


# --------------------------------------------------------------------------- JDS family


def check_jds_structure(A, J):
    n = A.n_rows
    lens = A.row_lengths()
    assert sorted(J.perm.tolist()) == list(range(n))
    assert np.array_equal(J.iperm[J.perm], np.arange(n))
    lp = lens[J.perm]
    assert np.all(np.diff(lp) <= 0)
    ties = np.diff(lp) == 0
    assert np.all(np.diff(J.perm)[ties] > 0)             # stable: equal lengths keep order
    for d in range(J.ndiag):
        assert J.jd_ptr[d + 1] - J.jd_ptr[d] == int((lens > d).sum())


@pytest.mark.parametrize("seed", range(5))
def test_jds_roundtrip_and_structure(seed):
    A, _ = rand_csr(200 + seed, n_rows=80, n_cols=80, density=0.1, long_rows=3, long_len=60)
    J = oracle.jds_from_csr(A)
    check_jds_structure(A, J)
    B = oracle.jds_to_csr(J, A.n_cols)
    assert np.array_equal(B.row_ptr, A.row_ptr)
    assert np.array_equal(B.col, A.col)
    assert np.array_equal(B.val, A.val)


@pytest.mark.parametrize("seed", range(5))
def test_jds_variants_bit_identical_to_crs(seed):
    """Paper Section 2: JDS, NUJDS, NBJDS and RBJDS keep each row's entries in CRS
    order, so in a serial evaluation every variant adds the same terms in the
    same order as CRS (NUJDS with unroll = Nj *is* CRS in the permuted basis,
    RBJDS with block size 1 is row by row, plain JDS is block size n)."""
    A, rng = rand_csr(300 + seed, n_rows=150, n_cols=150, density=0.06, long_rows=4, long_len=90)
    x = rng.uniform(-1, 1, A.n_cols)
    y0 = rng.uniform(-1, 1, A.n_rows)
    want = oracle.spmv_crs(A, x, y0, alpha=1.5, beta=-0.5)
    J = oracle.jds_from_csr(A)
    assert np.array_equal(oracle.spmv_jds(J, x, y0, 1.5, -0.5), want)
    for u in (1, 2, 4, J.ndiag):
        assert np.array_equal(oracle.spmv_nujds(J, x, u, y0, 1.5, -0.5), want)
    for b in (1, 7, 64, A.n_rows):
        assert np.array_equal(oracle.spmv_nbjds(J, x, b, y0, 1.5, -0.5), want)
    for C in (1, 8, 64, 256):
        B = oracle.blocked_from_jds(J, C)
        assert np.array_equal(oracle.spmv_blocked(B, x, y0, 1.5, -0.5), want)


def test_jds_symperm_is_permuted_problem():
    A, rng = rand_csr(400, n_rows=120, n_cols=120, density=0.08)
    x = rng.uniform(-1, 1, 120)
    y = oracle.spmv_crs(A, x)
    J = oracle.jds_from_csr(A, symperm=True)
    yp = oracle.spmv_jds(J, x[J.perm])          # x and y in the permuted basis
    assert np.array_equal(yp, y[J.perm])


def test_blocked_layout_rules():
    A, _ = rand_csr(500, n_rows=200, n_cols=200, density=0.05, long_rows=2, long_len=100)
    J = oracle.jds_from_csr(A)
    lens_p = A.row_lengths()[J.perm]
    for C in (1, 4, 64):
        B = oracle.blocked_from_jds(J, C)
        for s in range(B.n_slices):
            assert B.slice_nd[s] == lens_p[s * C]
            for rl in range(C):
                r = s * C + rl
                L = lens_p[r] if r < A.n_rows else 0
                for d in range(B.slice_nd[s]):
                    k = B.slice_ptr[s] + d * C + rl
                    if d < L:
                        assert B.bl_col[k] == J.jd_col[J.jd_ptr[d] + r]
                    else:
                        assert B.bl_col[k] == -1 and B.bl_val[k] == 0.0


def test_sojds_keeps_rows_and_is_close():
    A, rng = rand_csr(600, n_rows=300, n_cols=300, density=0.04, long_rows=3, long_len=40)
    x = rng.uniform(-1, 1, 300)
    J = oracle.jds_from_csr(A)
    want = oracle.spmv_crs(A, x)
    D = oracle.row_absdot(A, x)
    for C in (1, 8, 64, 300):
        B = oracle.blocked_from_jds(J, C, sojds=True)
        B0 = oracle.blocked_from_jds(J, C)
        assert np.array_equal(B.slice_ptr, B0.slice_ptr)
        for s in range(B.n_slices):
            for rl in range(C):
                ks = B.slice_ptr[s] + np.arange(B.slice_nd[s]) * C + rl
                a = sorted(zip(B.bl_col[ks].tolist(), B.bl_val[ks].tolist()))
                b = sorted(zip(B0.bl_col[ks].tolist(), B0.bl_val[ks].tolist()))
                assert a == b
        assert oracle.rel_err(oracle.spmv_blocked(B, x), want, D).max() <= 1e-13
    # the first row of a block keeps CRS order
    B = oracle.blocked_from_jds(J, 8, sojds=True)
    ks = B.slice_ptr[0] + np.arange(B.slice_nd[0]) * 8
    assert np.array_equal(B.bl_col[ks], J.jd_col[J.jd_ptr[:-1]])


def test_windowed_blocked_layout_brute_force():
    """Windowed RBJDS (rows sorted by decreasing length inside windows of sigma
    rows): every window's order and every slot rebuilt in Python from the
    definition; sigma >= n is the plain RBJDS of the JDS (pinned above); the
    blocked product stays bit-identical to CRS (each row summed in CRS
    order)."""
    A, rng = rand_csr(900, n_rows=300, n_cols=200, density=0.05, long_rows=4, long_len=90, empty=0.15)
    lens = A.row_lengths()
    x = rng.uniform(-1, 1, A.n_cols)
    for C, sigma in ((64, 64), (64, 128), (128, 128), (64, 320)):
        B = oracle.blocked_windowed(A, C, sigma)
        want_perm = []
        for w0 in range(0, A.n_rows, sigma):
            rows = range(w0, min(w0 + sigma, A.n_rows))
            want_perm += sorted(rows, key=lambda i: (-lens[i], i))
        assert B.perm.tolist() == want_perm
        for sl in range(B.n_slices):
            assert B.slice_nd[sl] == lens[want_perm[sl * C]]
            assert B.slice_ptr[sl + 1] - B.slice_ptr[sl] == B.slice_nd[sl] * C
            for rl in range(C):
                r = sl * C + rl
                row = want_perm[r] if r < A.n_rows else None
                for d in range(B.slice_nd[sl]):
                    k = B.slice_ptr[sl] + d * C + rl
                    if row is not None and d < lens[row]:
                        e = A.row_ptr[row] + d
                        assert B.bl_col[k] == A.col[e] and B.bl_val[k] == A.val[e]
                    else:
                        assert B.bl_col[k] == -1 and B.bl_val[k] == 0.0
        assert np.array_equal(oracle.spmv_blocked(B, x), oracle.spmv_crs(A, x))
    # one window of all rows is the paper's RBJDS
    for C in (64, 128):
        Bw = oracle.blocked_windowed(A, C, ((A.n_rows + C - 1) // C) * C)
        Bj = oracle.blocked_from_jds(oracle.jds_from_csr(A), C)
        assert np.array_equal(Bw.perm, Bj.perm) and np.array_equal(Bw.slice_ptr, Bj.slice_ptr)
        assert np.array_equal(Bw.bl_col, Bj.bl_col) and np.array_equal(Bw.bl_val, Bj.bl_val)
    with pytest.raises(ValueError):
        oracle.blocked_windowed(A, 64, 96)


def test_sojds_hand_worked_block():
    """The SOJDS slot rule on a block worked out by hand (paper Section 2,
    SOJDS: entries of each row re-sorted so the x access across the rows of a
    block is as close to stride one as possible; reading: the block's first
    row keeps CRS order, each next row fills slot d with its unused entry
    nearest to (previous row's column in slot d) + 1, the smaller column on a
    tie).  Six rows, C = 4, every row already in JDS order (lengths 3, 3, 3,
    2, 2, 2 keep their original order):

      row 0 {2, 5, 9}   first row of slice 0: CRS order        -> 2, 5, 9
      row 1 {0, 4, 10}  slot 0: want 2+1 = 3, |0-3|=3 |4-3|=1   -> 4
                        slot 1: want 5+1 = 6, |0-6|=6 |10-6|=4  -> 10
                        slot 2: only 0 left                     -> 0
      row 2 {1, 5, 11}  slot 0: want 4+1 = 5 (row 1's slot, not its CRS
                        order), |5-5|=0                          -> 5
                        slot 1: want 10+1 = 11                   -> 11
                        slot 2: only 1 left                      -> 1
      row 3 {4, 8}      slot 0: want 5+1 = 6, |4-6| = |8-6| = 2: tie,
                        smaller column                           -> 4
                        slot 1: want 11+1 = 12, only 8 left      -> 8
                        slot 2: beyond the row: padding          -> -1
      row 4 {3, 7}      first row of slice 1: CRS order          -> 3, 7
      row 5 {1, 4}      slot 0: want 3+1 = 4, |4-4| = 0          -> 4
                        slot 1: only 1 left                      -> 1
      rows 6, 7         do not exist: padding

    A rule without the "+1" (row 1 slot 0: |0-2| = |4-2|, tie -> 0), one that
    looks at the previous row's CRS order (row 2 slot 0: want 0+1 -> 1), or
    one that breaks ties upwards (row 3 slot 0 -> 8) fails this layout."""
    rows = [[2, 5, 9], [0, 4, 10], [1, 5, 11], [4, 8], [3, 7], [1, 4]]
    r = np.array([i for i, cs in enumerate(rows) for _ in cs], np.int32)
    c = np.array([cc for cs in rows for cc in cs], np.int32)
    v = 100.0 * r + c                              # each value names its entry
    A = oracle.csr_from_coo(6, 12, r, c, v)
    J = oracle.jds_from_csr(A)
    assert J.perm.tolist() == [0, 1, 2, 3, 4, 5]
    B = oracle.blocked_from_jds(J, 4, sojds=True)
    assert B.slice_ptr.tolist() == [0, 12, 20]
    assert B.slice_nd.tolist() == [3, 2]
    want_col = [2, 4, 5, 4,
                5, 10, 11, 8,
                9, 0, 1, -1,
                3, 4, -1, -1,
                7, 1, -1, -1]
    assert B.bl_col.tolist() == want_col
    rows_of_slot = [0, 1, 2, 3] * 3 + [4, 5, 6, 7] * 2
    want_val = [100.0 * rr + cc if cc >= 0 else 0.0 for rr, cc in zip(rows_of_slot, want_col)]
    assert B.bl_val.tolist() == want_val


def test_row_absdot_matches_python_floats():
    """D_i = sum_j |a_ij| |x_j| (the denominator of every tolerance) against a
    Python-float loop over a dense copy in ascending j: bit for bit on random
    patterns, exact on small integers, and never below |y_i|."""
    for seed in range(8):
        A, rng = rand_csr(700 + seed, n_rows=int(12 + 6 * seed), n_cols=int(64 - 4 * seed))
        x = rng.uniform(-1, 1, A.n_cols)
        M = dense_of(A)
        want = np.zeros(A.n_rows)
        for i in range(A.n_rows):
            s = 0.0
            for j in range(A.n_cols):
                if M[i, j] != 0.0:
                    s = s + abs(float(M[i, j])) * abs(float(x[j]))
            want[i] = s
        D = oracle.row_absdot(A, x)
        assert np.array_equal(D, want)
        assert np.all(np.abs(oracle.spmv_crs(A, x)) <= D * (1 + 1e-15))
    A, rng = rand_csr(720, n_rows=50, n_cols=60, integer=True)
    x = rng.integers(-8, 9, A.n_cols).astype(np.float64)
    M = dense_of(A).astype(np.int64)
    want = (np.abs(M) @ np.abs(x.astype(np.int64))).astype(np.float64)
    assert np.array_equal(oracle.row_absdot(A, x), want)


def test_jds_empty_rows_and_all_empty():
    A = oracle.csr_from_coo(5, 5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    J = oracle.jds_from_csr(A)
    assert J.ndiag == 0 and J.jd_ptr.tolist() == [0]
    y = oracle.spmv_jds(J, np.ones(5), np.full(5, 2.0), alpha=1.0, beta=0.5)
    assert y.tolist() == [1.0] * 5


# --------------------------------------------------------------------------- bf16


def test_bf16_matches_torch_on_float_inputs():
    """For inputs that are already floats, one RNE step from double equals
    torch's float -> bfloat16 conversion (also round-to-nearest-even)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(20000), rng.standard_normal(2000) * 1e-39,
                        rng.standard_normal(1000) * 1e38, [0.0, -0.0, 1.0, -2.5]])
    v = v.astype(np.float32).astype(np.float64)
    got = oracle.round_bf16_bits(v)
    want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_bf16_ties_and_double_rounding():
    one = 1.0
    cases = {
        one + 2.0 ** -8: 0x3F80,                 # tie -> even (1.0)
        one + 3 * 2.0 ** -8: 0x3F82,             # tie -> even (1 + 2^-6)
        one + 2.0 ** -8 + 2.0 ** -40: 0x3F81,    # just above the tie: up (a float would round first to the tie)
        -(one + 2.0 ** -8 + 2.0 ** -40): 0xBF81,
        2.0 ** -133: 0x0001,                     # smallest bf16 subnormal
        2.0 ** -134: 0x0000,                     # tie between 0 and 2^-133 -> even (0)
        3 * 2.0 ** -135: 0x0001,
        255 * 2.0 ** 120: 0x7F7F,                # largest finite
        511 * 2.0 ** 119: 0x7F80,                # halfway to 2^128 -> even -> infinity
        float("inf"): 0x7F80,
    }
    got = oracle.round_bf16_bits(np.array(list(cases.keys())))
    assert [int(g) for g in got] == list(cases.values())


# --------------------------------------------------------------------------- transpose / gradients


def test_transpose_matches_dense():
    A, rng = rand_csr(700, n_rows=40, n_cols=55, density=0.1)
    rowT, colT, tmap = oracle.transpose(A)
    T = oracle.CSR(A.n_cols, A.n_rows, rowT, colT, A.val[tmap])
    assert np.array_equal(dense_of(T), dense_of(A).T)
    assert np.all(np.diff(colT)[np.diff(T.row_index()) == 0] > 0)     # rows of A^T ascending
    g = rng.uniform(-1, 1, A.n_rows)
    assert np.allclose(oracle.spmv_crs_transposed(A, g), dense_of(A).T @ g, rtol=0, atol=1e-14)


def test_grad_vals_identities():
    A, rng = rand_csr(800, n_rows=60, n_cols=60, density=0.1)
    x = rng.uniform(-1, 1, 60)
    g = rng.uniform(-1, 1, 60)
    dv = oracle.grad_vals(A, g, x)
    y = oracle.spmv_crs(A, x)
    # y is linear in the values: sum_k val_k * dval_k = <g, A x>
    assert abs(np.dot(A.val, dv) - np.dot(g, y)) <= 1e-13 * np.abs(g).sum() * oracle.row_absdot(A, x).max()
    # adjoint: <g, A x> = <A^T g, x>
    assert abs(np.dot(oracle.spmv_crs_transposed(A, g), x) - np.dot(g, y)) <= 1e-13 * 60
    # central difference in one value (exact: the map is linear)
    k = 17
    e = 1e-3
    Ap = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
    Am = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
    Ap.val[k] += e
    Am.val[k] -= e
    fd = (np.dot(g, oracle.spmv_crs(Ap, x)) - np.dot(g, oracle.spmv_crs(Am, x))) / (2 * e)
    assert abs(fd - dv[k]) <= 1e-10


# --------------------------------------------------------------------------- Chebyshev


def test_chebyshev_closed_form_on_sine_modes():
    g = json.load(open(os.path.join(GOLD, "laplacian20.json")))
    A = lap()
    # A_s = (A - 6 I) / 6 on the same pattern
    vals = A.val / 6.0
    diag = A.row_index() == A.col
    vals[diag] = (A.val[diag] - 6.0) / 6.0
    As = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals)
    for e in g["chebyshev20"]:
        v = sine_mode(*e["mode"])
        ys = oracle.cheb_forward(As, v, 20)
        T20 = math.cos(20 * math.acos(e["lambda_s"]))
        assert abs(T20 - e["T20"]) <= 1e-13
        assert np.abs(ys[20] - T20 * v).max() <= 1e-11
        loss, dx, dval, _ = oracle.cheb_loss_grad(As, v, 20)
        assert abs(loss - T20 ** 2 * np.dot(v, v)) <= 1e-10 * np.dot(v, v)
        # A_s symmetric, v an eigenvector: grad_x = 2 T20(A_s)^T T20(A_s) v = 2 T20^2 v
        assert np.abs(dx - 2 * T20 ** 2 * v).max() <= 1e-10


def _small_c5(n=2000, seed=0):
    rng = np.random.default_rng(seed)
    r, c, v, nn, _ = synth.banded_uniform(n=n, band=50, dtype=np.float64)
    A = oracle.csr_from_coo(nn, nn, r, c, v)
    x = rng.uniform(-1, 1, nn)
    return A, x


def test_chebyshev_gradient_central_differences():
    A, x = _small_c5(400)
    steps = 20
    loss, dx, dval, _ = oracle.cheb_loss_grad(A, x, steps)
    rng = np.random.default_rng(9)
    eps = 1e-3

    def L(AA, xx):
        return float(np.sum(oracle.cheb_forward(AA, xx, steps)[steps] ** 2))

    # x: the loss is quadratic in x, so the central difference is exact up to rounding
    for i in rng.choice(A.n_rows, 12, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[i] += eps
        xm[i] -= eps
        fd = (L(A, xp) - L(A, xm)) / (2 * eps)
        assert abs(fd - dx[i]) <= 1e-8 * max(1.0, abs(loss))
    # vals: degree-40 polynomial, O(eps^2) truncation
    for k in rng.choice(A.nnz, 12, replace=False):
        Ap = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
        Am = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
        Ap.val[k] += eps
        Am.val[k] -= eps
        fd = (L(Ap, x) - L(Am, x)) / (2 * eps)
        assert abs(fd - dval[k]) <= 1e-5 * max(abs(fd), 1e-3 * abs(loss))


def test_chebyshev_directional_derivative():
    A, x = _small_c5(600, seed=2)
    steps = 20
    loss, dx, dval, _ = oracle.cheb_loss_grad(A, x, steps)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(A.n_rows)
    w = rng.standard_normal(A.nnz) * np.abs(A.val).mean()    # same scale as the values
    eps = 1e-4

    def L(vals, xx):
        AA = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals)
        return float(np.sum(oracle.cheb_forward(AA, xx, steps)[steps] ** 2))

    def fd(e):
        return (L(A.val + e * w, x + e * u) - L(A.val - e * w, x - e * u)) / (2 * e)

    an = np.dot(dx, u) + np.dot(dval, w)
    e1, e2 = abs(fd(eps) - an), abs(fd(eps / 2) - an)
    assert e1 <= 1e-6 * max(abs(an), abs(loss))
    # central differences converge at second order towards the adjoint value
    assert e2 <= 0.35 * e1 or e2 <= 1e-9 * abs(loss)


# --------------------------------------------------------------- one-triangle storage


def rand_sym(seed, n=48, density=0.12, integer=False, empty=0.1, long_rows=0, long_len=0):
    rng = np.random.default_rng(1000 + seed)
    r, c, v, n_, _ = synth.random_symmetric(n, density, rng, integer=integer, empty_rows=empty,
                                            long_rows=long_rows, long_len=long_len)
    return oracle.csr_from_coo(n_, n_, r, c, v), rng


@pytest.mark.parametrize("seed", range(5))
def test_csr_upper_brute_force(seed):
    """Upper triangle against a dense copy: the entries with col >= row, in
    ascending column order per row, and A = U + U^T - diag(U)."""
    A, _ = rand_sym(seed, n=20 + 7 * seed)
    M = dense_of(A)
    assert np.array_equal(M, M.T)
    U = oracle.csr_upper(A)
    want_rp = [0]
    want_c, want_v = [], []
    for i in range(A.n_rows):
        for j in range(A.n_cols):
            if j >= i and M[i, j] != 0.0:
                want_c.append(j)
                want_v.append(M[i, j])
        want_rp.append(len(want_c))
    assert np.array_equal(U.row_ptr, np.array(want_rp, np.int32))
    assert np.array_equal(U.col, np.array(want_c, np.int32))
    assert np.array_equal(U.val, np.array(want_v))
    MU = dense_of(U)
    assert np.array_equal(MU + MU.T - np.diag(np.diag(MU)), M)


def test_csr_upper_drops_lower_entries_unread():
    """Entries below the diagonal never reach U: changing them leaves U as is."""
    A, _ = rand_sym(7, n=30)
    rows = A.row_index()
    B = oracle.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.where(A.col < rows, 99.0, A.val))
    U, V = oracle.csr_upper(A), oracle.csr_upper(B)
    assert np.array_equal(U.val, V.val) and np.array_equal(U.col, V.col)


@pytest.mark.parametrize("seed", range(6))
def test_spmv_crs_sym_bit_identical_to_full_crs(seed):
    """Row i of the triangle product sums in ascending column order, as the
    full CRS product does on the symmetric matrix with sorted rows: the two
    are bit-identical for any values."""
    A, rng = rand_sym(seed, n=30 + 11 * seed, long_rows=2, long_len=25)
    U = oracle.csr_upper(A)
    x = rng.uniform(-1, 1, A.n_rows)
    y0 = rng.uniform(-1, 1, A.n_rows)
    for alpha, beta in ((1.0, 0.0), (-0.75, 0.5), (2.0, 1.0)):
        got = oracle.spmv_crs_sym(U, x, y0, alpha, beta)
        want = oracle.spmv_crs(A, x, y0, alpha, beta)
        assert np.array_equal(got, want)


def test_spmv_crs_sym_dense_and_integer():
    """Against dense Python floats (1e-14 of the row scale) and exactly on
    integer values, where every partial sum is exact."""
    A, rng = rand_sym(11, n=60, density=0.2)
    U = oracle.csr_upper(A)
    x = rng.uniform(-1, 1, A.n_rows)
    M = dense_of(A)
    want = np.array([sum(float(M[i, j]) * float(x[j]) for j in range(A.n_cols)) for i in range(A.n_rows)])
    scale = np.abs(M) @ np.abs(x)
    assert np.all(np.abs(oracle.spmv_crs_sym(U, x) - want) <= 1e-14 * np.maximum(scale, 1e-300))
    Ai, rng = rand_sym(12, n=60, density=0.2, integer=True)
    Ui = oracle.csr_upper(Ai)
    xi = synth.integer_vector(Ai.n_rows, rng)
    Mi = dense_of(Ai)
    assert np.array_equal(oracle.spmv_crs_sym(Ui, xi), Mi @ xi)


def test_spmv_crs_sym_beta_zero_ignores_y_and_empty():
    A, rng = rand_sym(13, n=25, empty=0.4)
    U = oracle.csr_upper(A)
    x = rng.uniform(-1, 1, A.n_rows)
    got = oracle.spmv_crs_sym(U, x, np.full(A.n_rows, np.nan), 1.0, 0.0)
    assert np.all(np.isfinite(got))
    E = oracle.CSR(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert oracle.csr_upper(E).nnz == 0
    assert np.array_equal(oracle.spmv_crs_sym(oracle.csr_upper(E), np.ones(5), np.ones(5), 1.0, 2.0), np.full(5, 2.0))
