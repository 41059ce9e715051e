"""Multi-vector (SpMM), many-matrix (batched persistent launch, HIP graph replay),
transposed products and value gradients on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import FP64_TOL, gpu_csr, max_err, rand_coo, to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")

U32, U64 = 2.0 ** -24, 2.0 ** -53


def gamma(k, u):
    return k * u / (1 - k * u)


def colmajor_from(X_np, dtype):
    """(n, k) numpy -> column-major device block."""
    t = torch.from_numpy(np.ascontiguousarray(X_np.T)).to("cuda").to(dtype)
    return t.t()


@pytest.mark.parametrize("k", [1, 3, 8, 11, 32, 40, 64])
def test_spmm_fp64(k):
    r, c, v, nr, nc, rng = rand_coo(60 + k, 6000, 5000, 0.002, empty_rows=0.1, long_rows=6, long_len=2000)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    X = rng.uniform(-1, 1, (nc, k))
    Y0 = rng.uniform(-1, 1, (nr, k))
    want = oracle.spmm_crs(R, X, alpha=1.5, beta=-0.5, Y=Y0)
    A = gpu_csr(sp, r, c, v, nr, nc)
    J = sp.jds_from_csr(A)
    Xd = colmajor_from(X, torch.float64)
    for name, fn in (("crs", lambda Y: sp.spmm_crs(A, Xd, Y, 1.5, -0.5)),
                     ("jds", lambda Y: sp.spmm_jds(J, Xd, Y, 1.5, -0.5)),
                     ("crs_colmajor", lambda Y: sp.spmm_crs(A, Xd, Y, 1.5, -0.5, interleave=False)),
                     ("jds_colmajor", lambda Y: sp.spmm_jds(J, Xd, Y, 1.5, -0.5, interleave=False))):
        got = to_np(fn(colmajor_from(Y0, torch.float64)))
        for j in range(k):
            D = 1.5 * oracle.row_absdot(R, X[:, j]) + 0.5 * np.abs(Y0[:, j])
            e = oracle.rel_err(got[:, j], want[:, j], D).max()
            assert e <= FP64_TOL, (name, j, e)


def test_spmm_integer_exact_and_fp32_bound():
    r, c, v, nr, nc, rng = rand_coo(70, 4000, 4000, 0.003, integer=True, long_rows=4, long_len=3000)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    k = 9
    X = rng.integers(-8, 9, (nc, k)).astype(np.float64)
    want = oracle.spmm_crs(R, X)
    A = gpu_csr(sp, r, c, v, nr, nc)
    J = sp.jds_from_csr(A)
    Xd = colmajor_from(X, torch.float64)
    for il in (True, False):
        assert np.array_equal(to_np(sp.spmm_crs(A, Xd, interleave=il)), want)
        assert np.array_equal(to_np(sp.spmm_jds(J, Xd, interleave=il)), want)
    # a long row (> 4096 entries) on the interleaved path, k > 64 falls back to column-major
    r2, c2, v2, nr, nc, _ = rand_coo(72, 300, 6000, 0.01, integer=True)
    rr = np.concatenate([r2, np.full(4500, 7, np.int32)])
    cc = np.concatenate([c2, rng.choice(nc, 4500, replace=False).astype(np.int32)])
    vv = np.concatenate([v2, rng.integers(-8, 9, 4500).astype(np.float64)])
    R2 = oracle.csr_from_coo(nr, nc, rr, cc, vv)
    A2 = gpu_csr(sp, rr, cc, vv, nr, nc)
    X2 = rng.integers(-8, 9, (nc, 70)).astype(np.float64)
    want2 = oracle.spmm_crs(R2, X2)
    assert np.array_equal(to_np(sp.spmm_crs(A2, colmajor_from(X2, torch.float64))), want2)
    assert np.array_equal(to_np(sp.spmm_crs(A2, colmajor_from(X2[:, :5], torch.float64))), want2[:, :5])
    assert np.array_equal(to_np(sp.spmm_jds(sp.jds_from_csr(A2), colmajor_from(X2[:, :17], torch.float64))),
                          want2[:, :17])
    # float32 values and vectors
    r, c, v, nr, nc, rng = rand_coo(71, 4000, 4000, 0.003)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    vq = oracle.round_f32(R.val).astype(np.float64)
    Rq = oracle.CSR(nr, nc, R.row_ptr, R.col, vq)
    X = rng.uniform(-1, 1, (nc, k)).astype(np.float32).astype(np.float64)
    want = oracle.spmm_crs(Rq, X)
    A = gpu_csr(sp, r, c, v, nr, nc, torch.float32)
    J = sp.jds_from_csr(A)
    Xd = colmajor_from(X, torch.float32)
    L = R.row_lengths()
    for got in (to_np(sp.spmm_crs(A, Xd)), to_np(sp.spmm_jds(J, Xd))):
        for j in range(k):
            D = oracle.row_absdot(Rq, X[:, j])
            assert np.all(np.abs(got[:, j] - want[:, j]) <= (gamma(L + 1, U32) + U32) * D)


_PAIRS = [(torch.float64, torch.float64), (torch.float32, torch.float32), (torch.float32, torch.float64),
          (torch.bfloat16, torch.float32), (torch.bfloat16, torch.float64), (torch.float64, torch.float32)]


@pytest.fixture(scope="module")
def mixed_spmm_matrix():
    """Rows of 1-80 entries (rows cross the entry shares of the 256- and
    1024-entry plan blocks), 10% empty rows, four single-row blocks of 2,000
    entries and two rows of 4,500 (FP64 accumulation for reduced values)."""
    rng = np.random.default_rng(77)
    n_rows, n_cols = 6000, 7000
    lens = rng.integers(1, 81, n_rows)
    lens[rng.random(n_rows) < 0.1] = 0
    lens[[5, 2100, 2101, 4999]] = 2000
    lens[[17, 3000]] = 4500
    r = np.repeat(np.arange(n_rows), lens).astype(np.int32)
    c = np.concatenate([rng.choice(n_cols, L, replace=False) for L in lens if L]).astype(np.int32)
    v = rng.standard_normal(len(r))
    return r, c, v, n_rows, n_cols, rng


@pytest.mark.parametrize("vdt,xdt", _PAIRS, ids=[f"{str(a)[6:]}-{str(b)[6:]}" for a, b in _PAIRS])
def test_spmm_every_dtype_pair(mixed_spmm_matrix, vdt, xdt):
    """Every value/vector pair that spmm_crs and spmm_jds export, on the
    interleaved and column-major paths, with the default and a 256-entry CRS
    plan: against the oracle on the rounded values and vectors, under the
    single-vector bound (x rounded to FP32, L+1 roundings for reduced values
    in rows of <= 4096 entries; FP64 products and sums otherwise; one more
    rounding for FP32 output)."""
    r, c, v, nr, nc, rng = mixed_spmm_matrix
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    if vdt == torch.float64:
        vq = R.val
    elif vdt == torch.float32:
        vq = oracle.round_f32(R.val).astype(np.float64)
    else:
        vq = oracle.bf16_bits_to_f64(oracle.round_bf16_bits(R.val))
    Rq = oracle.CSR(nr, nc, R.row_ptr, R.col, vq)
    L = R.row_lengths()
    A64 = gpu_csr(sp, r, c, v, nr, nc)
    A = A64 if vdt == torch.float64 else A64.with_values(sp.spmv_convert_values(A64.val, vdt))
    assert np.array_equal(to_np(A.val.to(torch.float64)), vq)
    J = sp.jds_from_csr(A)
    for k in (3, 8, 32, 64):
        X = rng.uniform(-1, 1, (nc, k))
        if xdt == torch.float32:
            X = X.astype(np.float32).astype(np.float64)
        want = oracle.spmm_crs(Rq, X)
        Xd = colmajor_from(X, xdt)
        wide = (L > 4096) | (vdt == torch.float64)
        u = np.where(wide, gamma(L + 1, U64), gamma(L + 1, U32)) + (U32 if xdt == torch.float32 else 0.0)
        runs = []
        for bn in (0, 256):
            A.plan = None
            sp.spmv_crs_plan(A, bn)
            runs += [(f"crs_il_b{bn}", to_np(sp.spmm_crs(A, Xd))),
                     (f"crs_cm_b{bn}", to_np(sp.spmm_crs(A, Xd, interleave=False)))]
        runs += [("jds_il", to_np(sp.spmm_jds(J, Xd))), ("jds_cm", to_np(sp.spmm_jds(J, Xd, interleave=False)))]
        for name, got in runs:
            for j in range(k):
                D = oracle.row_absdot(Rq, X[:, j])
                err = np.abs(got[:, j].astype(np.float64) - want[:, j])
                assert np.all(err <= u * D), (name, k, j, float(np.max(err / np.maximum(u * D, 1e-300))))
                assert np.all(got[L == 0, j] == 0), (name, k, j)


def small_batch(count, integer=False, seed=0):
    mats = []
    rng = np.random.default_rng(seed)
    for m in range(count):
        n = int(rng.integers(30, 3000))
        lengths = rng.integers(5, min(40, n) + 1, size=n)
        rows = np.repeat(np.arange(n), lengths)
        cols = np.concatenate([rng.choice(n, L, replace=False) for L in lengths])
        if integer:
            vals = rng.integers(-8, 9, len(rows)).astype(np.float64)
            x = rng.integers(-8, 9, n).astype(np.float64)
        else:
            vals = rng.standard_normal(len(rows)).astype(np.float32).astype(np.float64)
            x = rng.uniform(-1, 1, n).astype(np.float32).astype(np.float64)
        mats.append((rows.astype(np.int32), cols.astype(np.int32), vals, n, x))
    return mats


def build_batched(mats, Cs, **kw):
    blocked = []
    for i, (r, c, v, n, _) in enumerate(mats):
        A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v).to(torch.float32))
        blocked.append(sp.jds_blocked_from_jds(sp.jds_from_csr(A), Cs[i % len(Cs)]))
    return sp.Batched(blocked, **kw)


@pytest.mark.parametrize("rpw", [64, 16])
def test_batched_matches_oracle(rpw):
    mats = small_batch(40, seed=rpw)
    Bt = build_batched(mats, Cs=(64, 128, 256), rows_per_wave=rpw)
    x = torch.cat([to_dev(m[4]).to(torch.float32) for m in mats])
    y = to_np(Bt(x)).astype(np.float64)
    off = 0
    for r, c, v, n, xm in mats:
        R = oracle.csr_from_coo(n, n, r, c, v)
        want = oracle.spmv_crs(R, xm)
        D = oracle.row_absdot(R, xm)
        L = R.row_lengths()
        assert np.all(np.abs(y[off:off + n] - want) <= (gamma(L + 1, U32) + U32) * D)
        off += n


def test_batched_integer_exact_and_graph_replay():
    mats = small_batch(30, integer=True, seed=5)
    Bt = build_batched(mats, Cs=(64, 192))
    x = torch.cat([to_dev(m[4]).to(torch.float32) for m in mats])
    want = np.concatenate([oracle.spmv_crs(oracle.csr_from_coo(n, n, r, c, v), xm) for r, c, v, n, xm in mats])
    eager = Bt(x)
    assert np.array_equal(to_np(eager).astype(np.float64), want)
    y = torch.empty_like(eager)
    g = sp.Graph()
    with g.capture():
        Bt(x, y)
    for rep in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), rep
        other = Bt(x)                       # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(other, eager)


def test_graph_replay_of_single_matrix_kernels():
    r, c, v, nr, nc, rng = rand_coo(80, 20000, 20000, 0.001, long_rows=10, long_len=3000)
    A = gpu_csr(sp, r, c, v, nr, nc)
    J = sp.jds_from_csr(A)
    B = sp.jds_blocked_from_jds(J, 128)
    sp.spmv_crs_plan(A)
    x = to_dev(rng.uniform(-1, 1, nc))
    outs = [torch.empty(nr, dtype=torch.float64, device="cuda") for _ in range(3)]
    eager = [sp.spmv_crs(A, x), sp.spmv_jds(J, x), sp.spmv_jds_blocked(B, x)]
    g = sp.Graph()
    with g.capture():
        sp.spmv_crs(A, x, outs[0])
        sp.spmv_jds(J, x, outs[1])
        sp.spmv_jds_blocked(B, x, outs[2])
    for rep in range(3):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep


def test_graph_replay_of_split_dia_and_multivector_calls():
    """The other compute calls are capturable too: column and row split,
    DIA (full and symmetric), the staged CRS kernel and the interleaved multi-vector products
    (staging kernel + product) replay bit-identically to their eager runs,
    with eager work between the replays."""
    r, c, v, n, _, rng = rand_coo(81, 12000, 12000, 0.001, long_rows=6, long_len=2500)
    off = r != c                                                      # a symmetric matrix for DIA
    rs, cs, vs = np.concatenate([r, c[off]]), np.concatenate([c, r[off]]), np.concatenate([v, v[off]])
    A = gpu_csr(sp, rs, cs, vs, n, n)
    sp.spmv_crs_plan(A)
    J = sp.jds_from_csr(A)
    S, RS = sp.Split(A), sp.RowSplit(A)
    D, Ds = sp.dia_from_csr(A), sp.dia_from_csr(A, symmetric=True)
    x = to_dev(rng.uniform(-1, 1, n))
    X = colmajor_from(rng.uniform(-1, 1, (n, 8)), torch.float64)
    ws = sp.spmm_workspace(n, 8, torch.float64, "cuda")
    Ast = A.with_values(A.val)
    Ast.staged = True                                                 # the staged CRS kernel
    calls = [lambda y: sp.spmv_crs_split(S, x, y), lambda y: sp.spmv_jds_split(S, x, y),
             lambda y: sp.spmv_jds_row_split(RS, x, y), lambda y: sp.spmv_dia(D, x, y),
             lambda y: sp.spmv_dia(Ds, x, y), lambda y: sp.spmv_crs(Ast, x, y),
             lambda Y: sp.spmm_crs(A, X, Y, ws=ws), lambda Y: sp.spmm_jds(J, X, Y, ws=ws)]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(6)] + \
           [sp.colmajor(n, 8, torch.float64, "cuda") for _ in range(2)]
    eager = []
    for fn, o in zip(calls, outs):
        fn(o)
        eager.append(o.clone())
    g = sp.Graph()
    with g.capture():
        for fn, o in zip(calls, outs):
            fn(o)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), (rep, i)
        sp.spmv_crs(A, x)                                             # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("transpose", ["crs", "jds"])
def test_transposed_product_and_value_gradient(transpose):
    from paper_0910_4836_amd.autograd import SpMVOperator
    r, c, v, n, _, rng = rand_coo(90, 6000, 6000, 0.002, empty_rows=0.05, long_rows=5, long_len=1500)
    R = oracle.csr_from_coo(n, n, r, c, v)
    A = gpu_csr(sp, r, c, v, n, n)
    op = SpMVOperator(A, transpose=transpose)
    vals = op.J.jd_val
    g = rng.uniform(-1, 1, n)
    x = rng.uniform(-1, 1, n)
    # dx = A^T g
    want = oracle.spmv_crs_transposed(R, g)
    rowT, colT, tmap = oracle.transpose(R)
    RT = oracle.CSR(n, n, rowT, colT, R.val[tmap])
    DT = oracle.row_absdot(RT, g)
    assert max_err(op.rmatvec(vals, to_dev(g)), want, DT) <= FP64_TOL
    # dval in JDS order: oracle value gradient (CRS order) moved by the oracle's own JDS order
    dv_crs = oracle.grad_vals(R, g, x)
    Rpos = oracle.CSR(n, n, R.row_ptr, R.col, np.arange(R.nnz, dtype=np.float64))
    order = oracle.jds_from_csr(Rpos).jd_val.astype(np.int64)
    assert np.array_equal(to_np(op.jds_src).astype(np.int64), order)
    got = to_np(op.grad_vals(to_dev(g), to_dev(x)))
    assert np.array_equal(got, dv_crs[order])                      # one product each: bit-exact
    out = to_dev(np.ones(R.nnz))
    got2 = to_np(op.grad_vals(to_dev(g), to_dev(x), out, alpha=2.0, beta=1.0))
    assert np.allclose(got2, 2.0 * dv_crs[order] + 1.0, rtol=0, atol=4e-16)
    # values refreshed through the transpose map (A^T's CRS order, or its JDS order)
    want_vT = R.val[tmap]
    if transpose == "jds":
        want_vT = want_vT[oracle.jds_from_csr(oracle.CSR(n, n, rowT, colT, np.arange(R.nnz, dtype=np.float64)))
                          .jd_val.astype(np.int64)]
    assert np.array_equal(to_np(op.transposed_values(vals)), want_vT)


def test_autotuner_batched_and_cache(tmp_path):
    from paper_0910_4836_amd import autotune
    mats = small_batch(12, seed=9)
    jds = []
    for r, c, v, n, _ in mats:
        A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v).to(torch.float32))
        jds.append(sp.jds_from_csr(A))
    cache = str(tmp_path / "tune.json")
    tuner = autotune.Autotuner(cache, cs=(64, 128), rs=(64, 16), us=(2, 4))
    Bt = autotune.build_batched(jds, tuner)
    assert tuner.log and len(tuner.log[0]["timings_ms"]) == 8
    x = torch.cat([to_dev(m[4]).to(torch.float32) for m in mats])
    y = to_np(Bt(x)).astype(np.float64)
    off = 0
    for r, c, v, n, xm in mats:
        R = oracle.csr_from_coo(n, n, r, c, v)
        want = oracle.spmv_crs(R, xm)
        D = oracle.row_absdot(R, xm)
        assert np.all(np.abs(y[off:off + n] - want) <= (gamma(R.row_lengths() + 1, U32) + U32) * D)
        off += n
    # a second tuner reads the cached choice without timing anything
    t2 = autotune.Autotuner(cache, cs=(64, 128), rs=(64, 16), us=(2, 4))
    assert t2.tune_batched(jds) == (Bt.mats_C, Bt.rows_per_wave, Bt.unroll) and not t2.log
    # single-matrix tuning (JDS and blocked JDS): any choice computes the same y
    r, c, v, n, _, rng = rand_coo(95, 20000, 20000, 0.001, long_rows=10, long_len=3000)
    R = oracle.csr_from_coo(n, n, r, c, v)
    A = gpu_csr(sp, r, c, v, n, n)
    J = sp.jds_from_csr(A)
    xx = rng.uniform(-1, 1, n)
    xd = to_dev(xx)
    want, D = oracle.spmv_crs(R, xx), oracle.row_absdot(R, xx)
    U, mi, Wj = tuner.tune_jds(J, xd)
    assert Wj in autotune.W_CANDIDATES
    assert max_err(sp.spmv_jds(J, xd, unroll=U, max_iters=mi, wg_waves=Wj), want, D) <= FP64_TOL
    C_, R_, U2, Wb = tuner.tune_blocked(J, xd)
    B = sp.jds_blocked_from_jds(J, C_)
    assert max_err(sp.spmv_jds_blocked(B, xd, rows_per_wave=R_, unroll=U2, wg_waves=Wb), want, D) <= FP64_TOL
    bn = autotune.tune_crs(tuner, A, xd, J.ndiag)
    assert bn in autotune.BLOCK_NNZ_CANDIDATES + autotune.STAGED_BLOCK_NNZ_CANDIDATES and A.block_nnz == bn
    assert max_err(sp.spmv_crs(A, xd), want, D) <= FP64_TOL
    # class plan or XCD-local tile plan: a cached boolean, either launch the same y
    jt = tuner.tune_jds_launch(J, xd, U, mi, Wj)
    bt = tuner.tune_blocked_launch(B, xd, R_, U2, Wb)
    assert isinstance(jt, bool) and isinstance(bt, bool)
    assert max_err(sp.spmv_jds_tiled(J, xd, unroll=U, max_iters=mi, wg_waves=Wj), want, D) <= FP64_TOL
    assert max_err(sp.spmv_jds_blocked_tiled(B, xd, unroll=U2, rows_per_wave=R_, wg_waves=Wb), want, D) <= FP64_TOL
    t3 = autotune.Autotuner(cache, cs=(64, 128), rs=(64, 16), us=(2, 4))
    assert t3.tune_jds(J, xd) == (U, mi, Wj) and t3.tune_blocked(J, xd) == (C_, R_, U2, Wb) and not t3.log
    assert t3.tune_jds_launch(J, xd, U, mi, Wj) == jt and t3.tune_blocked_launch(B, xd, R_, U2, Wb) == bt
    assert not t3.log
    assert autotune.tune_crs(t3, A, xd, J.ndiag) == bn and not t3.log
    # the kernel choice (entry or row order) comes back from the cache too
    A2 = sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val)
    assert autotune.tune_crs(t3, A2, xd, J.ndiag) == bn and A2.staged == A.staged and not t3.log
    assert max_err(sp.spmv_crs(A2, xd), want, D) <= FP64_TOL
    # multi-vector CRS plan: its own copy of the structure, A's plan untouched
    Am = autotune.tune_spmm_crs(tuner, A, 8, torch.float64, J.ndiag)
    assert Am.block_nnz in (256, 512, 1024) and A.block_nnz == bn and Am.plan is not A.plan
    X = rng.uniform(-1, 1, (n, 8))
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda").t()
    Y = to_np(sp.spmm_crs(Am, Xd))
    want_X = oracle.spmm_crs(R, X)
    for j in range(8):
        assert oracle.rel_err(Y[:, j], want_X[:, j], oracle.row_absdot(R, X[:, j])).max() <= FP64_TOL
    t4 = autotune.Autotuner(cache)
    assert autotune.tune_spmm_crs(t4, A, 8, torch.float64, J.ndiag).block_nnz == Am.block_nnz and not t4.log


# ---- multi-vector products over blocked-JDS storage (global and windowed row order)


def _blocked_storages(A):
    """Blocked JDS at C = 64 and 256 (global length order) and windowed at
    C = 64 with windows of 512 and 4096 rows (square matrices only)."""
    J = sp.jds_from_csr(A)
    out = [("blocked_c64", sp.jds_blocked_from_jds(J, 64)), ("blocked_c256", sp.jds_blocked_from_jds(J, 256))]
    if A.n_rows == A.n_cols:
        out += [("windowed_s512", sp.jds_blocked_windowed_from_csr(A, 64, 512)),
                ("windowed_s4096", sp.jds_blocked_windowed_from_csr(A, 64, 4096))]
    return out


@pytest.mark.parametrize("k", [1, 3, 8, 11, 32, 40, 64])
def test_spmm_jds_blocked_fp64(k):
    r, c, v, n, _, rng = rand_coo(160 + k, 6000, 6000, 0.002, empty_rows=0.1, long_rows=6, long_len=2000)
    R = oracle.csr_from_coo(n, n, r, c, v)
    X = rng.uniform(-1, 1, (n, k))
    Y0 = rng.uniform(-1, 1, (n, k))
    want = oracle.spmm_crs(R, X, alpha=1.5, beta=-0.5, Y=Y0)
    A = gpu_csr(sp, r, c, v, n, n)
    Xd = colmajor_from(X, torch.float64)
    # both launch choices: lane groups per row (1 or up to 8) and records
    # dealt to XCD ranges of equal work or in turn
    for name, B in _blocked_storages(A):
        for mg, xr in ((0, None), (1, True), (8, False), (8, True)):
            got = to_np(sp.spmm_jds_blocked(B, Xd, colmajor_from(Y0, torch.float64), 1.5, -0.5, max_groups=mg,
                                            xcd_ranges=xr))
            for j in range(k):
                D = 1.5 * oracle.row_absdot(R, X[:, j]) + 0.5 * np.abs(Y0[:, j])
                e = oracle.rel_err(got[:, j], want[:, j], D).max()
                assert e <= FP64_TOL, (name, mg, xr, j, e)


def test_spmm_jds_blocked_rectangular_and_integer_exact():
    # rectangular, integer values, a row of 4,500 entries (FP64 accumulation
    # for reduced-precision values), every k from the single to the widest
    r, c, v, nr, nc, rng = rand_coo(171, 3000, 7000, 0.003, integer=True, empty_rows=0.2)
    rr = np.concatenate([r, np.full(4500, 11, np.int32)])
    cc = np.concatenate([c, rng.choice(nc, 4500, replace=False).astype(np.int32)])
    vv = np.concatenate([v, rng.integers(-8, 9, 4500).astype(np.float64)])
    R = oracle.csr_from_coo(nr, nc, rr, cc, vv)
    A = gpu_csr(sp, rr, cc, vv, nr, nc)
    for name, B in _blocked_storages(A):
        for vdt, xdt in ((torch.float64, torch.float64), (torch.float32, torch.float32),
                         (torch.bfloat16, torch.float64)):
            Bq = B if vdt == torch.float64 else B.with_values(sp.spmv_convert_values(B.bl_val, vdt))
            for k in (1, 5, 16, 64):
                X = rng.integers(-8, 9, (nc, k)).astype(np.float64)
                got = to_np(sp.spmm_jds_blocked(Bq, colmajor_from(X, xdt)))
                assert np.array_equal(got.astype(np.float64), oracle.spmm_crs(R, X)), (name, str(vdt), k)


@pytest.mark.parametrize("vdt,xdt", _PAIRS, ids=[f"{str(a)[6:]}-{str(b)[6:]}" for a, b in _PAIRS])
def test_spmm_jds_blocked_every_dtype_pair(mixed_spmm_matrix, vdt, xdt):
    """The single-vector bound on rounded inputs (see test_spmm_every_dtype_pair),
    for the blocked storages in both row orders (square part of the matrix)."""
    r0, c0, v0, nr, nc0, rng = mixed_spmm_matrix
    keep = c0 < nr
    # the rectangular matrix (rows of 4,500 entries: FP64 accumulation for
    # reduced values; global order only) and its square part (both orders)
    for r, c, v, nc in ((r0, c0, v0, nc0), (r0[keep], c0[keep], v0[keep], nr)):
        _check_blocked_pair(r, c, v, nr, nc, rng, vdt, xdt)


def _check_blocked_pair(r, c, v, nr, nc, rng, vdt, xdt):
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    if vdt == torch.float64:
        vq = R.val
    elif vdt == torch.float32:
        vq = oracle.round_f32(R.val).astype(np.float64)
    else:
        vq = oracle.bf16_bits_to_f64(oracle.round_bf16_bits(R.val))
    Rq = oracle.CSR(nr, nc, R.row_ptr, R.col, vq)
    L = R.row_lengths()
    A = gpu_csr(sp, r, c, v, nr, nc)
    for name, B in _blocked_storages(A):
        Bq = B if vdt == torch.float64 else B.with_values(sp.spmv_convert_values(B.bl_val, vdt))
        for k in (3, 8, 32, 64):
            X = rng.uniform(-1, 1, (nc, k))
            if xdt == torch.float32:
                X = X.astype(np.float32).astype(np.float64)
            want = oracle.spmm_crs(Rq, X)
            wide = (L > 4096) | (vdt == torch.float64)
            u = np.where(wide, gamma(L + 1, U64), gamma(L + 1, U32)) + (U32 if xdt == torch.float32 else 0.0)
            got = to_np(sp.spmm_jds_blocked(Bq, colmajor_from(X, xdt)))
            for j in range(k):
                D = oracle.row_absdot(Rq, X[:, j])
                err = np.abs(got[:, j].astype(np.float64) - want[:, j])
                assert np.all(err <= u * D), (name, k, j, float(np.max(err / np.maximum(u * D, 1e-300))))


def test_spmm_jds_blocked_edge_cases():
    """A matrix smaller than one slice, a matrix of empty rows (beta*Y only,
    NaN in Y ignored at beta = 0), and n = 0 / k = 0 calls that launch nothing."""
    rng = np.random.default_rng(181)
    # 40 rows: one partial slice of the 64-row height
    r, c, v, n, _, _ = rand_coo(182, 40, 40, 0.2, empty_rows=0.2)
    R = oracle.csr_from_coo(n, n, r, c, v)
    A = gpu_csr(sp, r, c, v, n, n)
    for name, B in _blocked_storages(A):
        for k in (1, 6, 33):
            X = rng.uniform(-1, 1, (n, k))
            got = to_np(sp.spmm_jds_blocked(B, colmajor_from(X, torch.float64)))
            want = oracle.spmm_crs(R, X)
            for j in range(k):
                assert oracle.rel_err(got[:, j], want[:, j], oracle.row_absdot(R, X[:, j])).max() <= FP64_TOL, name
    # every row empty
    n = 300
    E = sp.CSR(n, n, torch.zeros(n + 1, dtype=torch.int32, device="cuda"),
               torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.float64, device="cuda"))
    for name, B in _blocked_storages(E):
        X = colmajor_from(rng.uniform(-1, 1, (n, 4)), torch.float64)
        Y0 = rng.uniform(-1, 1, (n, 4))
        got = to_np(sp.spmm_jds_blocked(B, X, colmajor_from(Y0, torch.float64), 1.0, 0.5))
        assert np.array_equal(got, 0.5 * Y0), name
        Yn = colmajor_from(np.full((n, 4), np.nan), torch.float64)
        assert np.array_equal(to_np(sp.spmm_jds_blocked(B, X, Yn, 1.0, 0.0)), np.zeros((n, 4))), name
