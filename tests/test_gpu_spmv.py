"""GPU SpMV (CRS, JDS, blocked JDS) against the FP64 oracle.

FP64 kernels: max_i |y_i - y_ref_i| / sum_j |a_ij||x_j| <= 1e-12 (two summation
orders of an L-term row differ by at most about 2*L*2^-53 relative to that
scale: 4.4e-13 at L = 2000).  Integer-valued inputs: bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import FP64_TOL, gpu_csr, max_err, rand_coo, to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")


def all_forms(A, rows_per_wave=(0,), unrolls=(0,), Cs=(64,), symperm=False, max_iters=(0,), split=True, waves=(0,)):
    """Yields (name, fn(x, y, alpha, beta)) for every kernel variant on matrix A."""
    yield "crs", lambda x, y, a, b: sp.spmv_crs(A, x, y, a, b)
    yield "crs_wave", lambda x, y, a, b: sp.spmv_crs(A, x, y, a, b, use_plan=False)
    for bn in (256, 4096):
        Ab = sp.spmv_crs_plan(sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val), bn)
        yield f"crs_b{bn}", (lambda Ab=Ab: lambda x, y, a, b: sp.spmv_crs(Ab, x, y, a, b))()
    # the staged kernel (gathers in row order) over plans of every block size
    for bn in (256, 1024, 4096):
        As = sp.spmv_crs_plan(sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val), bn)
        As.staged = True
        yield f"crs_staged_b{bn}", (lambda As=As: lambda x, y, a, b: sp.spmv_crs(As, x, y, a, b))()
    if split and not symperm:
        S = sp.Split(A)
        w = waves[-1]
        yield "crs_split", lambda x, y, a, b: sp.spmv_crs_split(S, x, y, a, b)
        yield "jds_split", lambda x, y, a, b: sp.spmv_jds_split(S, x, y, a, b, wg_waves=w)
        yield "blocked_split", lambda x, y, a, b: sp.spmv_jds_blocked_split(S, x, y, a, b, C_=Cs[-1], wg_waves=w)
        RS = sp.RowSplit(A)
        yield "jds_row_split", lambda x, y, a, b: sp.spmv_jds_row_split(RS, x, y, a, b, max_iters=max_iters[-1],
                                                                        wg_waves=w)
        yield "blocked_row_split", lambda x, y, a, b: sp.spmv_jds_blocked_row_split(
            RS, x, y, a, b, C_=Cs[-1], rows_per_wave=rows_per_wave[-1], max_iters=max_iters[-1], wg_waves=w)
    J = sp.jds_from_csr(A, symperm=symperm)
    for u in unrolls:
        for mi in max_iters:
            for w in waves:
                yield f"jds_u{u}_mi{mi}_w{w}", (lambda J=J, u=u, mi=mi, w=w:
                                                lambda x, y, a, b: sp.spmv_jds(J, x, y, a, b, u, mi, w))()
    # the XCD-local tile plan
    for R in rows_per_wave:
        for w in waves:
            yield f"jds_tiled_R{R}_w{w}", (lambda J=J, R=R, w=w: lambda x, y, a, b: sp.spmv_jds_tiled(
                J, x, y, a, b, max_iters=max_iters[-1], rows_per_wave=R, wg_waves=w))()
    for C in Cs:
        B = sp.jds_blocked_from_jds(J, C)
        for R in rows_per_wave:
            for mi in max_iters:
                for w in waves:
                    yield f"blk_C{C}_R{R}_mi{mi}_w{w}", (lambda B=B, R=R, mi=mi, w=w:
                                                         lambda x, y, a, b: sp.spmv_jds_blocked(B, x, y, a, b, R, 0,
                                                                                                mi, w))()
        # the tile-plan launch, on the plain order and on windowed orders
        # (windows of one slice, four slices, and one window of all rows)
        yield f"blk_tiled_C{C}", (lambda B=B: lambda x, y, a, b: sp.spmv_jds_blocked_tiled(
            B, x, y, a, b, max_iters=max_iters[-1], wg_waves=waves[-1]))()
        if symperm:
            continue
        for sg in (C, 4 * C, A.n_rows + C):
            Bw = sp.jds_blocked_windowed_from_csr(A, C, sg)
            for R in rows_per_wave:
                for w in waves:
                    yield f"win_C{C}_s{sg}_R{R}_w{w}", (lambda Bw=Bw, R=R, w=w: lambda x, y, a, b:
                                                       sp.spmv_jds_blocked_tiled(Bw, x, y, a, b,
                                                                                 max_iters=max_iters[-1],
                                                                                 rows_per_wave=R, wg_waves=w))()


def run_case(r, c, v, nr, nc, x, y0=None, alpha=1.0, beta=0.0, exact=False, **kw):
    A = gpu_csr(sp, r, c, v, nr, nc)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    want = oracle.spmv_crs(R, x, y0, alpha, beta)
    D = oracle.row_absdot(R, x) * abs(alpha)
    if y0 is not None:
        D = D + abs(beta) * np.abs(y0)
    xd = to_dev(x)
    for name, fn in all_forms(A, **kw):
        y = to_dev(y0.copy()) if y0 is not None else None
        got = fn(xd, y, alpha, beta)
        if exact:
            assert np.array_equal(to_np(got), want), name
        else:
            e = max_err(got, want, D)
            assert e <= FP64_TOL, f"{name}: {e:.3e}"


def test_laplacian_all_kernels_and_sine_mode():
    r, c, v, n, _ = synth.laplacian3d(20)
    x = synth.uniform_vector(n, synth.rng_for(1, 1))
    run_case(r, c, v, n, n, x, unrolls=(2, 4, 8), Cs=(64, 256), rows_per_wave=(0, 8, 16, 64))
    # closed form: A v = lambda v for the (3, 7, 11) sine mode
    m = 20
    idx = np.arange(n)
    i, j, k = idx % m, (idx // m) % m, idx // (m * m)
    vmode = np.sin(3 * np.pi * (i + 1) / 21) * np.sin(7 * np.pi * (j + 1) / 21) * np.sin(11 * np.pi * (k + 1) / 21)
    lam = 6 - 2 * np.cos(3 * np.pi / 21) - 2 * np.cos(7 * np.pi / 21) - 2 * np.cos(11 * np.pi / 21)
    A = gpu_csr(sp, r, c, v, n, n)
    R = oracle.csr_from_coo(n, n, r, c, v)
    D = oracle.row_absdot(R, vmode)
    for name, fn in all_forms(A):
        got = fn(to_dev(vmode), None, 1.0, 0.0)
        assert max_err(got, lam * vmode, D) <= FP64_TOL, name


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_ragged_with_empty_and_long_rows(seed):
    # rows: many short, some empty, a few long (multi-class split, ragged tails)
    r, c, v, nr, nc, rng = rand_coo(10 + seed, 9000 + 37 * seed, 7000, 0.0015, empty_rows=0.25, long_rows=40,
                                    long_len=3000)
    x = rng.uniform(-1, 1, nc)
    run_case(r, c, v, nr, nc, x, unrolls=(2, 8), Cs=(64, 128), rows_per_wave=(0, 16, 64), max_iters=(0, 4),
             waves=(0, 4, 8))


def test_alpha_beta_accumulate():
    r, c, v, nr, nc, rng = rand_coo(20, 3000, 3000, 0.004, empty_rows=0.1, long_rows=5, long_len=900)
    x = rng.uniform(-1, 1, nc)
    y0 = rng.uniform(-1, 1, nr)
    run_case(r, c, v, nr, nc, x, y0, alpha=-1.75, beta=0.5)
    run_case(r, c, v, nr, nc, x, None, alpha=2.0, beta=0.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_integer_bit_exact(seed):
    r, c, v, nr, nc, rng = rand_coo(30 + seed, 4000, 4000, 0.003, integer=True, empty_rows=0.1, long_rows=8,
                                    long_len=2500)
    x = synth.integer_vector(nc, rng)
    y0 = synth.integer_vector(nr, rng)
    run_case(r, c, v, nr, nc, x, exact=True, unrolls=(2, 4, 8), Cs=(64, 256), rows_per_wave=(0, 8, 32),
             max_iters=(0, 2), waves=(0, 4))
    run_case(r, c, v, nr, nc, x, y0, alpha=1.0, beta=1.0, exact=True)     # the paper's accumulate form


def test_symperm_mode():
    r, c, v, n, _, rng = rand_coo(40, 5000, 5000, 0.002, empty_rows=0.1, long_rows=10, long_len=500)
    x = rng.uniform(-1, 1, n)
    R = oracle.csr_from_coo(n, n, r, c, v)
    want = oracle.spmv_crs(R, x)
    D = oracle.row_absdot(R, x)
    A = gpu_csr(sp, r, c, v, n, n)
    J = sp.jds_from_csr(A, symperm=True)
    perm = to_np(J.perm)
    xp = sp.spmv_permute_vec(J.perm, to_dev(x))
    yp = sp.spmv_jds(J, xp)
    y = sp.spmv_permute_vec(J.perm, yp, inverse=True)
    assert max_err(y, want, D) <= FP64_TOL
    B = sp.jds_blocked_from_jds(J, 128)
    yb = sp.spmv_jds_blocked(B, xp)
    assert max_err(yb, want[perm], D[perm]) <= FP64_TOL
    for w in (4, 8):
        yw = sp.spmv_jds(J, xp, max_iters=4, wg_waves=w)
        assert max_err(yw, want[perm], D[perm]) <= FP64_TOL
        yw = sp.spmv_jds_blocked(B, xp, rows_per_wave=16, max_iters=4, wg_waves=w)
        assert max_err(yw, want[perm], D[perm]) <= FP64_TOL


def test_empty_matrix_and_single_row():
    x = to_dev(np.ones(5))
    A = sp.csr_from_coo(4, 5, to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0)))
    y0 = to_dev(np.full(4, 3.0))
    for name, fn in all_forms(A):
        got = fn(x, y0.clone(), 1.0, 0.5)
        assert to_np(got).tolist() == [1.5] * 4, name
    # n = 1, one dense row of 5000 entries (a single long row)
    nc = 5000
    r = np.zeros(nc, np.int32)
    c = np.arange(nc, dtype=np.int32)
    vv = np.random.default_rng(1).standard_normal(nc)
    xx = np.random.default_rng(2).uniform(-1, 1, nc)
    run_case(r, c, vv, 1, nc, xx)


@pytest.mark.parametrize("block_nnz", [256, 1024, 4096])
def test_blocks_of_many_short_rows(block_nnz):
    """Rows of 0-3 entries (blocks of up to 2048 rows, one lane per row) mixed
    with runs of 17-entry rows (the 256-row cap), runs of mixed lengths up to
    700 and a few rows longer than any block."""
    rng = np.random.default_rng(70 + block_nnz)
    nr, nc = 30000, 20000
    lens = rng.integers(0, 4, nr)
    lens[10000:11000] = 17                      # a run of rows just above "short"
    lens[21000:21030] = rng.integers(4, 40, 30)
    # blocks mixing row lengths on both sides of every power of two up to 700
    lens[20000:20240] = rng.choice([8, 9, 16, 17, 32, 33, 64, 65, 128, 129, 256, 257, 700], 240)
    lens[rng.choice(nr, 5, replace=False)] = 5000
    r = np.repeat(np.arange(nr, dtype=np.int32), lens)
    c = np.concatenate([rng.choice(nc, L, replace=False) for L in lens]).astype(np.int32)
    v = rng.standard_normal(len(r))
    x = rng.uniform(-1, 1, nc)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    want = oracle.spmv_crs(R, x)
    D = oracle.row_absdot(R, x)
    A = sp.spmv_crs_plan(gpu_csr(sp, r, c, v, nr, nc), block_nnz)
    plan = to_np(A.plan)
    sizes = np.diff(plan)
    if block_nnz >= 1024:
        assert sizes.max() > 256                  # the many-short-row path is taken
    rp = to_np(A.row_ptr)
    for b in np.nonzero(sizes > 256)[0]:          # ... only for blocks of short rows
        assert np.diff(rp[plan[b]:plan[b + 1] + 1]).max() <= 16 and sizes[b] <= 2048
    multi = sizes > 1
    assert np.all(rp[plan[1:]][multi] - rp[plan[:-1]][multi] <= block_nnz)
    assert max_err(sp.spmv_crs(A, to_dev(x)), want, D) <= FP64_TOL
    As = A.with_values(A.val)
    As.staged = True
    assert max_err(sp.spmv_crs(As, to_dev(x)), want, D) <= FP64_TOL
    X = rng.uniform(-1, 1, (nc, 9))
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda").t()        # column-major (n, k)
    want_X = oracle.spmm_crs(R, X)
    for il in (True, False):
        Y = to_np(sp.spmm_crs(A, Xd, interleave=il))
        for j in range(9):
            e = oracle.rel_err(Y[:, j], want_X[:, j], oracle.row_absdot(R, X[:, j])).max()
            assert e <= FP64_TOL, (il, j, e)
    # integer values: bit-exact
    vi = rng.integers(-8, 9, len(r)).astype(np.float64)
    xi = synth.integer_vector(nc, rng)
    Ai = sp.spmv_crs_plan(gpu_csr(sp, r, c, vi, nr, nc), block_nnz)
    want_i = oracle.spmv_crs(oracle.csr_from_coo(nr, nc, r, c, vi), xi)
    assert np.array_equal(to_np(sp.spmv_crs(Ai, to_dev(xi))), want_i)
    Ai.staged = True
    assert np.array_equal(to_np(sp.spmv_crs(Ai, to_dev(xi))), want_i)


def test_split_structure_is_a_column_partition():
    """Every part holds exactly the entries of its column range, in CRS order,
    over the rows that have one of them; slots are numbered row by row, part
    by part."""
    r, c, v, nr, nc, _ = rand_coo(60, 3000, 5000, 0.004, empty_rows=0.1, long_rows=4, long_len=3000)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    S = sp.Split(gpu_csr(sp, r, c, v, nr, nc))
    width = -(-(-(-nc // 8)) // 64) * 64
    rows = R.row_index()
    part = R.col // width
    present = np.zeros((nr, 8), dtype=bool)
    present[rows, part] = True
    slot_ptr = np.concatenate([[0], np.cumsum(present.sum(1))])
    assert np.array_equal(to_np(S.slot_ptr), slot_ptr)
    assert S.n_slots == present.sum()
    for k in range(8):
        Pk = S.parts[k]
        sel = part == k
        rk = np.nonzero(present[:, k])[0]
        assert Pk.n_rows == len(rk)
        cnt = np.bincount(rows[sel], minlength=nr)[rk]
        assert np.array_equal(to_np(Pk.row_ptr), np.concatenate([[0], np.cumsum(cnt)]))
        assert np.array_equal(to_np(Pk.col_idx), R.col[sel])
        assert np.array_equal(to_np(Pk.val), R.val[sel])
        want_dest = slot_ptr[rk] + present[rk, :k].sum(1)
        assert np.array_equal(to_np(S.part_dest(k)), want_dest)


@pytest.mark.parametrize("n_cols", [100, 64 * 8 * 3 + 5])
def test_split_narrow_and_empty_parts(n_cols):
    """Parts with no entries at all (few columns) and rows with no entries."""
    r, c, v, nr, nc, rng = rand_coo(61, 2000, n_cols, 0.02, empty_rows=0.3, long_rows=3, long_len=90)
    run_case(r, c, v, nr, nc, rng.uniform(-1, 1, nc), Cs=(64,))
    y0 = rng.uniform(-1, 1, nr)
    run_case(r, c, v, nr, nc, rng.uniform(-1, 1, nc), y0, alpha=0.5, beta=-2.0)


@pytest.mark.parametrize("case", ["random", "few_rows", "one_heavy_row", "no_entries"])
def test_row_split_structure(case):
    """Part k is rows [b_k, b_k+1) with b_k the first row whose row pointer
    reaches ceil(k*nnz/8) (k*n/8 without entries); its row pointer is the
    original one rebased to 0 and its entries are the original arrays from
    row_ptr[b_k] on."""
    rng = np.random.default_rng(62)
    if case == "random":
        r, c, v, nr, nc, _ = rand_coo(62, 5000, 4000, 0.003, empty_rows=0.2, long_rows=5, long_len=2000)
    elif case == "few_rows":                           # fewer rows than parts
        nr, nc = 3, 50
        r = np.repeat(np.arange(nr, dtype=np.int32), [7, 0, 20])
        c = np.concatenate([rng.choice(nc, 7, replace=False), rng.choice(nc, 20, replace=False)]).astype(np.int32)
        v = rng.standard_normal(len(r))
    elif case == "one_heavy_row":                      # one row holds almost every entry
        nr, nc = 1000, 3000
        lens = np.ones(nr, np.int64)
        lens[500] = 2900
        r = np.repeat(np.arange(nr, dtype=np.int32), lens)
        c = np.concatenate([rng.choice(nc, L, replace=False) for L in lens]).astype(np.int32)
        v = rng.standard_normal(len(r))
    else:
        nr, nc = 37, 10
        r = c = np.zeros(0, np.int32)
        v = np.zeros(0)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    RS = sp.RowSplit(gpu_csr(sp, r, c, v, nr, nc))
    nnz = R.nnz
    want_b = [0] + [int(np.searchsorted(R.row_ptr, -(-k * nnz // 8), side="left")) if nnz else k * nr // 8
                    for k in range(1, 8)] + [nr]
    assert RS.bounds.tolist() == want_b
    assert RS.entry_bounds.tolist() == [int(R.row_ptr[b]) for b in want_b]
    for k in range(8):
        a, b = want_b[k], want_b[k + 1]
        Pk = RS.parts[k]
        assert Pk.n_rows == b - a
        assert np.array_equal(to_np(Pk.row_ptr), R.row_ptr[a:b + 1] - R.row_ptr[a])
        e0, e1 = R.row_ptr[a], R.row_ptr[b]
        assert np.array_equal(to_np(Pk.col_idx), R.col[e0:e1])
        assert np.array_equal(to_np(Pk.val), R.val[e0:e1])
    # products through every part, including the empty ones
    x = rng.uniform(-1, 1, nc)
    y0 = rng.uniform(-1, 1, nr)
    want = oracle.spmv_crs(R, x, y0, 0.5, -1.5)
    D = 0.5 * oracle.row_absdot(R, x) + 1.5 * np.abs(y0)
    for C_ in (64, 128):
        got = sp.spmv_jds_blocked_row_split(RS, to_dev(x), to_dev(y0.copy()), 0.5, -1.5, C_=C_)
        assert max_err(got, want, D) <= FP64_TOL
    got = sp.spmv_jds_row_split(RS, to_dev(x), to_dev(y0.copy()), 0.5, -1.5)
    assert max_err(got, want, D) <= FP64_TOL


def test_row_split_rejects_bad_bounds():
    r, c, v, nr, nc, rng = rand_coo(63, 200, 200, 0.02)
    RS = sp.RowSplit(gpu_csr(sp, r, c, v, nr, nc))
    x = to_dev(rng.uniform(-1, 1, nc))
    RS.jds_parts()
    good = RS.bounds.copy()
    for bad in ([0, 10, 5, 30, 40, 50, 60, 70, nr], [1] + good[1:].tolist(), good[:-1].tolist() + [nr - 1]):
        RS.bounds = np.array(bad, dtype=np.int64)
        with pytest.raises(sp.SpmvError):
            sp.spmv_jds_row_split(RS, x)
        with pytest.raises(sp.SpmvError):
            sp.spmv_jds_blocked_row_split(RS, x)
    RS.bounds = good


def test_deterministic_repeat():
    r, c, v, nr, nc, rng = rand_coo(50, 20000, 20000, 0.001, long_rows=20, long_len=5000)
    x = to_dev(rng.uniform(-1, 1, nc))
    A = gpu_csr(sp, r, c, v, nr, nc)
    for name, fn in all_forms(A, max_iters=(0, 8)):
        a = to_np(fn(x, None, 1.0, 0.0))
        b = to_np(fn(x, None, 1.0, 0.0))
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("g", [0, 2, 3])
def test_row_shard_local_then_remote(g):
    """One GPU's share of a row-partitioned product over 4 GPUs: rows of shard
    g, local block (own columns, own slice of x) then remote block (other
    columns, whole x) accumulated with beta = 1, in CRS and JDS, equals those
    rows of the oracle's product."""
    G = 4
    r, c, v, nr, nc, rng = rand_coo(50 + g, 6000, 6000, 0.003, empty_rows=0.1, long_rows=6, long_len=2000)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    x = rng.uniform(-1, 1, nc)
    r0, r1 = g * nr // G, (g + 1) * nr // G
    want = oracle.spmv_crs(R, x)[r0:r1]
    D = oracle.row_absdot(R, x)[r0:r1]
    sel = (r >= r0) & (r < r1)
    rr, cc, vv = (r[sel] - r0).astype(np.int32), c[sel], v[sel]
    loc = (cc >= r0) & (cc < r1)
    m = r1 - r0
    AL = gpu_csr(sp, rr[loc], (cc[loc] - r0).astype(np.int32), vv[loc], m, m)
    AR = gpu_csr(sp, rr[~loc], cc[~loc], vv[~loc], m, nc)
    xd = to_dev(x)
    y = sp.spmv_crs(AL, xd[r0:r1])
    sp.spmv_crs(AR, xd, y, beta=1.0)
    assert max_err(y, want, D) <= FP64_TOL
    JL, JR = sp.jds_from_csr(AL), sp.jds_from_csr(AR)
    y = sp.spmv_jds(JL, xd[r0:r1])
    sp.spmv_jds(JR, xd, y, beta=1.0)
    assert max_err(y, want, D) <= FP64_TOL


def tile_rows(tiles, nt):
    """Rows covered by each record of a tile plan (first row, row count)."""
    T = to_np(tiles[:2 * nt]).reshape(-1, 2).astype(np.int64)
    return T[:, 0], T[:, 1] >> 8


@pytest.mark.parametrize("symperm", [False, True])
def test_xcd_local_tile_plans(symperm):
    """Long runs of one row length (here 1, 2 and 3 entries, over 10,000 rows
    each) are cut into XCD pieces, walked by place in their run, the rest
    dealt: every row is covered by exactly one record, blocked records stay
    inside one slice, and the tiled launches agree with the oracle (FP64,
    FP32 values, FP32 vectors)."""
    rng = np.random.default_rng(41)
    n = 60000
    lengths = rng.choice([0, 1, 2, 3, 5], size=n, p=[0.05, 0.3, 0.3, 0.3, 0.05])
    lengths[rng.choice(n, 30, replace=False)] = rng.integers(100, 3000, 30)      # rows beyond max_iters
    rows = np.repeat(np.arange(n), lengths).astype(np.int32)
    cols = np.concatenate([rng.choice(n, L, replace=False) for L in lengths if L]).astype(np.int32)
    vals = rng.standard_normal(len(rows))
    R = oracle.csr_from_coo(n, n, rows, cols, vals)
    A = gpu_csr(sp, rows, cols, vals, n, n)
    J = sp.jds_from_csr(A, symperm=symperm)
    x = rng.uniform(-1, 1, n)
    xp = x[to_np(J.perm)] if symperm else x
    want = oracle.spmv_crs(R, x)
    D = oracle.row_absdot(R, x)
    unperm = (lambda y: y[np.argsort(to_np(J.perm))]) if symperm else (lambda y: y)
    lens = np.diff(J.h_jd_ptr)
    rl = np.searchsorted(-lens, -np.arange(n), side="left")      # length of the r-th sorted row
    for mi, rpw, w in ((0, 0, 0), (32, 0, 4), (64, 16, 8)):
        tiles, nt, h_plan = sp.spmv_jds_tiles(J, mi, rpw, w)
        r0, cnt = tile_rows(tiles, nt)
        cover = np.zeros(n, np.int64)
        np.add.at(cover, np.concatenate([np.arange(a, a + m) for a, m in zip(r0, cnt)]), 1)
        assert (cover == 1).all() and h_plan[0] == 0 and h_plan[8] == nt
        # pieces (rows up to max_iters long, in runs of >= 1,024 of one
        # length): XCD k holds the k-th eighth of each run and walks its
        # pieces by their place in the run
        Lr = rl[r0]
        start, end = np.searchsorted(-rl, -Lr, side="left"), np.searchsorted(-rl, -Lr, side="right")
        place = (r0 - start) / (end - start)
        piece = (Lr <= (mi or 32)) & (end - start >= 1024)
        assert piece.sum() >= 8 * 5                  # five short lengths, each cut in 8
        for k in range(8):
            p, e = place[h_plan[k]:h_plan[k + 1]], (end - start)[h_plan[k]:h_plan[k + 1]]
            sel = piece[h_plan[k]:h_plan[k + 1]]
            assert np.all(np.diff(p[sel]) >= 0), (mi, rpw, w, k)
            assert np.all(p[sel] > k / 8 - 1 / e[sel]) and np.all(p[sel] < (k + 1) / 8), (mi, rpw, w, k)
        got = unperm(to_np(sp.spmv_jds_tiled(J, to_dev(xp), max_iters=mi, rows_per_wave=rpw, wg_waves=w)))
        assert oracle.rel_err(got, want, D).max() <= FP64_TOL, (mi, rpw, w)
        for C in (64, 256):
            B = sp.jds_blocked_from_jds(J, C)
            tiles, nt, h_plan = sp.spmv_jds_blocked_tiles(B, mi, rpw, w)
            r0, cnt = tile_rows(tiles, nt)
            assert np.all(r0 // C == (r0 + cnt - 1) // C)                     # inside one slice
            cover = np.zeros(n, np.int64)
            np.add.at(cover, np.concatenate([np.arange(a, a + m) for a, m in zip(r0, cnt)]), 1)
            assert (cover == 1).all()
            got = unperm(to_np(sp.spmv_jds_blocked_tiled(B, to_dev(xp), max_iters=mi, rows_per_wave=rpw,
                                                         wg_waves=w)))
            assert oracle.rel_err(got, want, D).max() <= FP64_TOL, (C, mi, rpw, w)
    # FP32 values with FP64 and FP32 vectors, against the oracle on the
    # rounded values and vectors: gamma_{L+1}(2^-24) D (+ 2^-24 D for FP32 y)
    Jq = J.with_values(sp.spmv_convert_values(J.jd_val, torch.float32))
    Rq = oracle.CSR(n, n, R.row_ptr, R.col, oracle.round_f32(R.val).astype(np.float64))
    u = 2.0 ** -24
    for f32x in (False, True):
        xq = oracle.round_f32(x).astype(np.float64) if f32x else x
        wq, Dq = oracle.spmv_crs(Rq, xq), oracle.row_absdot(Rq, xq)
        L = Rq.row_lengths() + 1
        lim = (L * u / (1 - L * u)) * Dq + (u * Dq if f32x else 0)
        xd = to_dev((xq[to_np(J.perm)] if symperm else xq).astype(np.float32 if f32x else np.float64))
        got = unperm(to_np(sp.spmv_jds_tiled(Jq, xd)).astype(np.float64))
        assert np.all(np.abs(got - wq) <= lim), f32x


def test_caller_plan_with_more_rows_than_the_planner_makes():
    """A caller's plan may hold more than 2,048 rows in one block (the planner
    never does): both CRS kernels accept any plan whose multi-row blocks stay
    within block_nnz entries; the staged kernel walks rows past 2,048 in its
    tail loop.  Rows of 0-2 entries, blocks of 3,000 and 2,000 rows."""
    rng = np.random.default_rng(77)
    nr, nc = 5000, 3000
    lens = rng.integers(0, 3, nr)
    assert lens[:3000].sum() <= 4096 and lens[3000:].sum() <= 4096
    r = np.repeat(np.arange(nr, dtype=np.int32), lens)
    c = np.concatenate([rng.choice(nc, L, replace=False) for L in lens]).astype(np.int32)
    v = rng.standard_normal(len(r))
    x = rng.uniform(-1, 1, nc)
    y0 = rng.uniform(-1, 1, nr)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    want = oracle.spmv_crs(R, x, y0, 1.5, -0.25)
    D = 1.5 * oracle.row_absdot(R, x) + 0.25 * np.abs(y0)
    A = gpu_csr(sp, r, c, v, nr, nc)
    A.plan = torch.tensor([0, 3000, nr], dtype=torch.int32, device="cuda")
    A.n_blocks, A.block_nnz = 2, 4096
    for staged in (False, True):
        A.staged = staged
        got = sp.spmv_crs(A, to_dev(x), to_dev(y0.copy()), 1.5, -0.25)
        assert max_err(got, want, D) <= FP64_TOL, staged
