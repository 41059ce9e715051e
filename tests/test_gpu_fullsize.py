"""Parity at the full workload sizes, in the configurations bench.py times.

The oracle cannot run every product at these sizes within a test, so each
check takes a seeded sample of rows (and of matrices for the many-matrix
form), builds the oracle's CRS of just those rows and compares row by row
with the same error measures as the small tests:
  FP64:  |y_i - y_ref_i| / D_i <= 1e-12,  D_i = sum_j |a_ij| |x_j|
  FP32 values / vectors: the accumulation bound gamma_{L+1}(2^-24) D_i
      (+ 2^-24 D_i when y is FP32) against the oracle run on the stored
      (rounded) values and vectors.
Structure properties that hold at any size (permutation, sorted lengths,
slot partition) are checked on the whole matrix.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import FP64_TOL, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
sp = pytest.importorskip("paper_0910_4836_amd")

U32 = 2.0 ** -24
N_SAMPLE = 4000


def gamma(k, u):
    return k * u / (1 - k * u)


def sample_rows(R: oracle.CSR, rows):
    """The oracle CRS of rows `rows` of R (all columns kept)."""
    lens = R.row_lengths()[rows]
    starts = R.row_ptr[rows].astype(np.int64)
    idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(lens.sum())
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return oracle.CSR(len(rows), R.n_cols, rp, R.col[idx], R.val[idx])


def coo_rows(n, r, c, v, rows):
    """The oracle CRS of rows `rows` of the COO matrix (r, c, v): only their
    triplets go through the oracle's COO -> CRS, so the test never sorts the
    whole matrix on the host."""
    keep = np.zeros(n, dtype=bool)
    keep[rows] = True
    sel = keep[r]
    return sample_rows(oracle.csr_from_coo(n, n, r[sel], c[sel], np.asarray(v[sel], np.float64)), rows)


def pick(n, seed, extra=()):
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(n, min(n, N_SAMPLE), replace=False), np.asarray(extra, np.int64)]))
    return rows.astype(np.int64)


@pytest.fixture(scope="module")
def powerlaw():
    r, c, v, n, _ = synth.powerlaw()
    x = synth.uniform_vector(n, synth.rng_for(2, 1))
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    return (r, c, v, n), A, x


def test_powerlaw_every_form_sampled(powerlaw):
    (r, c, v, n), A, x = powerlaw
    L = np.bincount(r, minlength=n)
    nnz = len(r)
    rows = pick(n, 11, extra=np.argsort(-L)[:50])            # plus the 50 longest rows
    sub = coo_rows(n, r, c, v, rows)
    want = oracle.spmv_crs(sub, x)
    D = oracle.row_absdot(sub, x)
    J = sp.jds_from_csr(A)
    B = sp.jds_blocked_from_jds(J, 64)
    S = sp.Split(A)
    xd = to_dev(x)
    # the launch parameters bench.py times come from the autotuner
    import tempfile
    from paper_0910_4836_amd import autotune
    tuner = autotune.Autotuner(cache_path=tempfile.mktemp(suffix=".json"))
    ju, jm, jw = tuner.tune_jds(J, xd)
    bC, bR, bU, bW = tuner.tune_blocked(J, xd)
    Bt = sp.jds_blocked_from_jds(J, bC)
    RS = sp.RowSplit(A)
    At = sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val)
    autotune.tune_crs(tuner, At, xd, J.ndiag)
    wS, wC, wU, wW = tuner.tune_windowed(A, xd, J.ndiag)
    BW = sp.jds_blocked_windowed_from_csr(A, wC, wS)
    forms = {"crs": lambda: sp.spmv_crs(A, xd), "jds": lambda: sp.spmv_jds(J, xd),
             "blocked": lambda: sp.spmv_jds_blocked(B, xd), "crs_split": lambda: sp.spmv_crs_split(S, xd),
             "jds_split": lambda: sp.spmv_jds_split(S, xd), "blocked_split": lambda: sp.spmv_jds_blocked_split(S, xd),
             "crs_tuned": lambda: sp.spmv_crs(At, xd),
             "jds_tuned": lambda: sp.spmv_jds(J, xd, unroll=ju, max_iters=jm, wg_waves=jw),
             "blocked_tuned": lambda: sp.spmv_jds_blocked(Bt, xd, rows_per_wave=bR, unroll=bU, wg_waves=bW),
             "jds_row_split": lambda: sp.spmv_jds_row_split(RS, xd, unroll=ju, max_iters=jm, wg_waves=jw),
             "blocked_row_split": lambda: sp.spmv_jds_blocked_row_split(RS, xd, C_=bC, rows_per_wave=bR, unroll=bU,
                                                                        wg_waves=bW),
             "blocked_windowed": lambda: sp.spmv_jds_blocked_tiled(BW, xd, unroll=wU, max_iters=32, wg_waves=wW)}
    for name, fn in forms.items():
        got = to_np(fn())[rows]
        e = oracle.rel_err(got, want, D).max()
        assert e <= FP64_TOL, f"{name}: {e:.3e}"
    # structure at full size: perm is a permutation sorting lengths down, ties by index
    perm = to_np(J.perm)[:n].astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    Lp = L[perm]
    assert np.all(np.diff(Lp) <= 0)
    same = np.diff(Lp) == 0
    assert np.all(np.diff(perm)[same] > 0)
    assert J.ndiag == L.max() and int(to_np(J.jd_ptr)[J.ndiag]) == nnz
    assert B.padded >= nnz
    # windowed order: each window of sigma rows is a permutation of itself,
    # sorted by length down, ties by index
    pw = to_np(BW.perm)[:n].astype(np.int64)
    assert np.array_equal(pw // BW.sigma, np.arange(n) // BW.sigma)
    Lw = L[pw]
    inside = (np.arange(1, n) % BW.sigma) != 0
    assert np.all(np.diff(Lw)[inside] <= 0)
    assert np.all(np.diff(pw)[inside & (np.diff(Lw) == 0)] > 0)
    # slots: one per (row, part) pair present
    assert S.n_slots == int(to_np(S.slot_ptr)[-1]) and S.n_slots <= min(nnz, 8 * n)
    # row parts: contiguous, each within one row of nnz/8 entries
    eb = RS.entry_bounds
    assert eb[0] == 0 and eb[-1] == nnz and np.all(np.diff(RS.bounds) >= 0)
    assert np.all(np.abs(eb[1:-1] - np.arange(1, 8) * nnz / 8) <= L.max())


def test_powerlaw_fp32_values_sampled(powerlaw):
    (r, c, v, n), A, x = powerlaw
    rows = pick(n, 12)
    sub = coo_rows(n, r, c, oracle.round_f32(v).astype(np.float64), rows)
    want = oracle.spmv_crs(sub, x)
    D = oracle.row_absdot(sub, x)
    lim = np.where(sub.row_lengths() > 4096, gamma(sub.row_lengths() + 1, 2.0 ** -53),
                   gamma(sub.row_lengths() + 1, U32)) * D
    A32 = A.with_values(sp.spmv_convert_values(A.val, torch.float32))
    A32.plan = None
    J32 = sp.jds_from_csr(A32)
    B32 = sp.jds_blocked_from_jds(J32, 64)
    xd = to_dev(x)
    for name, fn in (("crs", lambda: sp.spmv_crs(A32, xd)), ("jds", lambda: sp.spmv_jds(J32, xd)),
                     ("blocked", lambda: sp.spmv_jds_blocked(B32, xd))):
        got = to_np(fn())[rows]
        assert np.all(np.abs(got - want) <= lim), name


def test_powerlaw_multi_vector_sampled(powerlaw):
    (r, c, v, n), A, x = powerlaw
    rows = pick(n, 13)
    sub = coo_rows(n, r, c, v, rows)
    J = sp.jds_from_csr(A)
    # the plan bench.py times for the multi-vector CRS product (256-entry blocks)
    A256 = sp.spmv_crs_plan(sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val), 256)
    # and the blocked-JDS multi-vector product in both row orders (the window
    # sizes the suite line times; the global order with its launch default)
    B = sp.jds_blocked_from_jds(J, 64)
    wins = {sig: sp.jds_blocked_windowed_from_csr(A, 64, sig) for sig in (8192, 32768)}
    for k in (8, 32):
        X = np.random.default_rng(k).uniform(-1, 1, (n, k))
        Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda").t()
        for name, fn in (("crs", lambda: sp.spmm_crs(A, Xd)), ("crs_b256", lambda: sp.spmm_crs(A256, Xd)),
                         ("jds", lambda: sp.spmm_jds(J, Xd)), ("blocked", lambda: sp.spmm_jds_blocked(B, Xd)),
                         ("windowed_8192", lambda: sp.spmm_jds_blocked(wins[8192], Xd)),
                         ("windowed_32768", lambda: sp.spmm_jds_blocked(wins[32768], Xd))):
            Y = to_np(fn())
            for j in (0, k // 2, k - 1):
                want = oracle.spmv_crs(sub, X[:, j])
                e = oracle.rel_err(Y[rows, j], want, oracle.row_absdot(sub, X[:, j])).max()
                assert e <= FP64_TOL, (name, k, j, e)
        del Xd


def test_symmetric_diagonals_sampled():
    r, c, v, n, _ = synth.sym_diagonals()
    x = synth.uniform_vector(n, synth.rng_for(3, 1))
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    rows = pick(n, 14, extra=[0, 1, n // 2, n - 2, n - 1])
    sub = coo_rows(n, r, c, v, rows)
    del r, c, v
    want = oracle.spmv_crs(sub, x)
    D = oracle.row_absdot(sub, x)
    J = sp.jds_from_csr(A)
    B = sp.jds_blocked_from_jds(J, 64)
    xd = to_dev(x)
    # plus the launch configurations the autotuner picks for this matrix
    import tempfile
    from paper_0910_4836_amd import autotune
    tuner = autotune.Autotuner(cache_path=tempfile.mktemp(suffix=".json"))
    ju, jm, jw = tuner.tune_jds(J, xd)
    bC, bR, bU, bW = tuner.tune_blocked(J, xd)
    Bt = sp.jds_blocked_from_jds(J, bC)
    # CRS as the bench runs it (autotuned plan and kernel), and the staged
    # kernel at the block sizes the autotuner picks from on this matrix
    At = sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val)
    autotune.tune_crs(tuner, At, xd, J.ndiag)
    staged = {}
    for bn in (2048, 4096):
        staged[bn] = sp.spmv_crs_plan(sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val), bn)
        staged[bn].staged = True
    for name, fn in (("crs_tuned", lambda: sp.spmv_crs(At, xd)),
                     ("crs_staged_2048", lambda: sp.spmv_crs(staged[2048], xd)),
                     ("crs_staged_4096", lambda: sp.spmv_crs(staged[4096], xd)),
                     ("crs", lambda: sp.spmv_crs(A, xd)), ("jds", lambda: sp.spmv_jds(J, xd)),
                     ("blocked", lambda: sp.spmv_jds_blocked(B, xd)),
                     ("jds_tuned", lambda: sp.spmv_jds(J, xd, unroll=ju, max_iters=jm, wg_waves=jw)),
                     ("blocked_tuned", lambda: sp.spmv_jds_blocked(Bt, xd, rows_per_wave=bR, unroll=bU,
                                                                   wg_waves=bW))):
        e = oracle.rel_err(to_np(fn())[rows], want, D).max()
        assert e <= FP64_TOL, f"{name}: {e:.3e}"
    del Bt
    # the DIA + CRS hybrid: every entry of this matrix lies on one of its 25 diagonals
    Dd = sp.dia_from_csr(A)
    assert Dd.ndia == 25 and Dd.rem.nnz == 0
    e = oracle.rel_err(to_np(sp.spmv_dia(Dd, xd))[rows], want, D).max()
    assert e <= FP64_TOL, f"dia: {e:.3e}"
    del Dd
    # one-triangle CRS: the diagonal and one of each mirrored pair
    S = sp.csr_upper_from_csr(A)
    assert S.nnz == (A.nnz + n) // 2
    e = oracle.rel_err(to_np(sp.spmv_crs_sym(S, xd))[rows], want, D).max()
    assert e <= FP64_TOL, f"crs_sym: {e:.3e}"
    del S
    # reduced-precision values on the same rows
    for vdt in (torch.float32, torch.bfloat16):
        if vdt == torch.float32:
            vq = oracle.round_f32(sub.val).astype(np.float64)
        else:
            vq = oracle.bf16_bits_to_f64(oracle.round_bf16_bits(sub.val))
        subq = oracle.CSR(sub.n_rows, n, sub.row_ptr, sub.col, vq)
        wq = oracle.spmv_crs(subq, x)
        lim = gamma(subq.row_lengths() + 1, U32) * oracle.row_absdot(subq, x)
        Jq = J.with_values(sp.spmv_convert_values(J.jd_val, vdt))
        Bq = B.with_values(sp.spmv_convert_values(B.bl_val, vdt))
        Aq = staged[4096].with_values(sp.spmv_convert_values(A.val, vdt))
        for name, fn in (("jds", lambda: sp.spmv_jds(Jq, xd)), ("blocked", lambda: sp.spmv_jds_blocked(Bq, xd)),
                         ("crs_staged", lambda: sp.spmv_crs(Aq, xd))):
            assert np.all(np.abs(to_np(fn())[rows] - wq) <= lim), (vdt, name)


def test_hamiltonian_shaped_dia_sampled():
    """The Hamiltonian-shaped matrix (n = 6 M): the DIA hybrid with its
    remainder in CRS, in window-sorted slices and over one triangle of the
    diagonals, and CRS, on sampled rows against the oracle; the window-sorted
    forms bit-identical to the CRS-remainder forms on every row."""
    r, c, v, n, _ = synth.heavy_diagonals_band()
    x = synth.uniform_vector(n, synth.rng_for(6, 1))
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    rows = pick(n, 16, extra=[0, 1, 255, 256, n // 2, n - 257, n - 1])
    sub = coo_rows(n, r, c, v, rows)
    del r, c, v
    want = oracle.spmv_crs(sub, x)
    D = oracle.row_absdot(sub, x)
    xd = to_dev(x)
    e = oracle.rel_err(to_np(sp.spmv_crs(A, xd))[rows], want, D).max()
    assert e <= FP64_TOL, f"crs: {e:.3e}"
    for bn in (2048, 4096):                          # the staged CRS kernel
        As = sp.spmv_crs_plan(sp.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val), bn)
        As.staged = True
        e = oracle.rel_err(to_np(sp.spmv_crs(As, xd))[rows], want, D).max()
        assert e <= FP64_TOL, f"crs staged {bn}: {e:.3e}"
        del As
    for sym in (False, True):
        Dc = sp.dia_from_csr(A, symmetric=sym)
        Ds = sp.dia_from_csr(A, symmetric=sym, sliced=True)
        assert Dc.ndia == (7 if sym else 13) and Dc.rem.nnz > 0
        # window-sorted padding stays small on this matrix
        assert Ds.rem_slices.bl_col.numel() <= 1.1 * Ds.rem.nnz
        yc, ys = sp.spmv_dia(Dc, xd), sp.spmv_dia(Ds, xd)
        assert torch.equal(yc, ys), f"sym={sym}: sliced remainder differs from the CRS remainder"
        e = oracle.rel_err(to_np(ys)[rows], want, D).max()
        assert e <= FP64_TOL, f"dia sym={sym}: {e:.3e}"
        del Dc, Ds, yc, ys


def test_chebyshev_operator_sampled():
    """The banded + uniform FP32 operator: forward and transposed products."""
    from paper_0910_4836_amd import autograd as AG
    r, c, v, n, _ = synth.banded_uniform()
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    op = AG.SpMVOperator(A)
    vals = op.J.jd_val
    x = synth.uniform_vector(n, synth.rng_for(5, 1), np.float32)
    xd = to_dev(x)
    rows = pick(n, 15, extra=[0, n - 1])
    sub = coo_rows(n, r, c, v, rows)
    xx = x.astype(np.float64)
    want = oracle.spmv_crs(sub, xx)
    lim = (gamma(sub.row_lengths() + 1, U32) + U32) * oracle.row_absdot(sub, xx)
    got = to_np(op.matvec(vals, xd)).astype(np.float64)[rows]
    assert np.all(np.abs(got - want) <= lim)
    # A^T g on sampled rows of A^T (the triplets with their roles swapped)
    subT = coo_rows(n, c, r, v, rows)
    wT = oracle.spmv_crs(subT, xx)
    limT = (gamma(subT.row_lengths() + 1, U32) + U32) * oracle.row_absdot(subT, xx)
    gotT = to_np(op.rmatvec(vals, xd)).astype(np.float64)[rows]
    assert np.all(np.abs(gotT - wT) <= limT)


def test_many_matrices_sampled():
    """All 512 matrices in one persistent launch; a seeded sample of matrices
    (the largest and smallest among them) is checked against the oracle."""
    dev = torch.device("cuda", 0)
    mats, xs, host = [], [], []
    sizes = synth.many_matrix_sizes()
    rng = np.random.default_rng(16)
    check = set(rng.choice(len(sizes), 6, replace=False).tolist()) | {int(np.argmax(sizes)), int(np.argmin(sizes))}
    for m, (r, c, v, n, x) in enumerate(synth.many_matrices()):
        A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
        mats.append(sp.jds_blocked_from_jds(sp.jds_from_csr(A), 64))
        xs.append(to_dev(x))
        host.append((r, c, v, n, x) if m in check else None)
        del A
    Bt = sp.Batched(mats)
    y = to_np(Bt(torch.cat(xs)))
    for m in sorted(check):
        r, c, v, n, x = host[m]
        R = oracle.csr_from_coo(n, n, r, c, v.astype(np.float64))
        xx = x.astype(np.float64)
        want = oracle.spmv_crs(R, xx)
        lim = (gamma(R.row_lengths() + 1, U32) + U32) * oracle.row_absdot(R, xx)
        got = y[Bt.row_base[m]:Bt.row_base[m] + n].astype(np.float64)
        assert np.all(np.abs(got - want) <= lim), m


@pytest.mark.timeout(900)
def test_chebyshev_loss_and_gradient_full_size():
    """The full differentiable workload: n = 4,000,000, 80 M entries (16
    banded + 4 uniform per row, scaled to norm_inf = 1), 20-step Chebyshev
    recurrence, loss = ||y_20||^2, backward with a checkpoint every 5 steps,
    the operator's JDS launch taken from the autotuner as the benchmark does.
      FP32 on the GPU against the FP64 oracle (same FP32-rounded values):
          loss, y_20, dx, dvals within 2e-3 norm-wise (the FP32 recurrence
          bound of the small tests).
      FP64 on the GPU (same values): loss, dx, dvals within 1e-10 of the
          oracle, and a directional derivative <dx, u> + <dvals, w> for
          seeded directions supported on a 2,000-row slice (u on x's slice,
          w on those rows' entries) against central differences of the GPU
          FP64 loss: exact for u (the loss is quadratic in x), Richardson-
          extrapolated from eps = 1e-3 and 5e-4 for w (error O(eps^4));
          both within 1e-6 of sum |u_i dx_i| (resp. |w_e dval_e|)."""
    from paper_0910_4836_amd import autograd as AG
    from paper_0910_4836_amd import autotune
    import tempfile
    import os

    def say(msg):
        print(f"[c5 full] {msg}", flush=True)

    r, c, v, n, _ = synth.banded_uniform()
    assert n == 4_000_000 and len(r) == 80_000_000
    x32 = synth.uniform_vector(n, synth.rng_for(5, 1), np.float32)
    x64 = x32.astype(np.float64)
    say("generated")
    R = oracle.csr_from_coo(n, n, r, c, v.astype(np.float64))
    loss_ref, dx_ref, dval_ref, ys = oracle.cheb_loss_grad(R, x64, 20)
    y20_ref = ys[20].copy()
    del ys
    say(f"oracle loss {loss_ref:.6e}")

    def rel_inf(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    # FP32 operator, autotuned JDS launch
    A32 = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    op = AG.SpMVOperator(A32)
    xd32 = to_dev(x32)
    tuner = autotune.Autotuner(cache_path=os.path.join(tempfile.mkdtemp(), "autotune.json"))
    op.unroll, op.max_iters, op.wg_waves = tuner.tune_jds(op.J, xd32)
    order = to_np(op.jds_src).astype(np.int64)          # JDS slot -> CRS position
    vals = op.J.jd_val.clone().requires_grad_(True)
    xt = xd32.clone().requires_grad_(True)
    loss = AG.chebyshev_loss(op, vals, xt, steps=20, checkpoint=5)
    loss.backward()
    say(f"fp32 loss {loss.item():.6e}")
    assert abs(loss.item() - loss_ref) <= 2e-3 * abs(loss_ref)
    assert rel_inf(to_np(xt.grad).astype(np.float64), dx_ref) <= 2e-3
    assert rel_inf(to_np(vals.grad).astype(np.float64), dval_ref[order]) <= 2e-3
    y20 = AG.cheb_states(op, vals.detach(), xd32, 20)[20]
    assert rel_inf(to_np(y20).astype(np.float64), y20_ref) <= 2e-3
    del A32, op, vals, xt, y20
    torch.cuda.empty_cache()

    # FP64 operator over the same values
    A64 = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v.astype(np.float64)))
    op64 = AG.SpMVOperator(A64)
    op64.unroll, op64.max_iters, op64.wg_waves = tuner.tune_jds(op64.J, to_dev(x64))
    assert np.array_equal(to_np(op64.jds_src).astype(np.int64), order)
    v64 = op64.J.jd_val.clone()
    xd64 = to_dev(x64)
    vals = v64.clone().requires_grad_(True)
    xt = xd64.clone().requires_grad_(True)
    loss = AG.chebyshev_loss(op64, vals, xt, steps=20, checkpoint=5)
    loss.backward()
    dx64 = to_np(xt.grad)
    dv64 = to_np(vals.grad)
    say(f"fp64 loss {loss.item():.15e}")
    assert abs(loss.item() - loss_ref) <= 1e-10 * abs(loss_ref)
    assert rel_inf(dx64, dx_ref) <= 1e-10
    assert rel_inf(dv64, dval_ref[order]) <= 1e-10
    del vals, xt

    # directions on a 2,000-row slice
    rng = np.random.default_rng(20091031)
    r0 = int(rng.integers(0, n - 2000))
    u = np.zeros(n)
    u[r0:r0 + 2000] = rng.uniform(-1, 1, 2000)
    w_crs = np.zeros(R.nnz)
    a, b = int(R.row_ptr[r0]), int(R.row_ptr[r0 + 2000])
    w_crs[a:b] = rng.standard_normal(b - a) * np.abs(R.val[a:b])   # relative changes of the slice's values
    w = w_crs[order]
    ud, wd = to_dev(u), to_dev(w)

    def loss64(tx, tv):
        with torch.no_grad():
            return AG.chebyshev_loss(op64, v64 + tv * wd, xd64 + tx * ud, steps=20, checkpoint=20).item()

    fd_x = (loss64(1e-3, 0.0) - loss64(-1e-3, 0.0)) / 2e-3

    def fd_v(e):
        return (loss64(0.0, e) - loss64(0.0, -e)) / (2 * e)
    fd_w = (4 * fd_v(5e-4) - fd_v(1e-3)) / 3
    dd_x, dd_w = float(np.dot(dx64, u)), float(np.dot(dv64, w))
    say(f"directional: x {dd_x:.9e} vs FD {fd_x:.9e}; vals {dd_w:.9e} vs FD {fd_w:.9e}")
    assert abs(dd_x - fd_x) <= 1e-6 * float(np.abs(dx64 * u).sum())
    assert abs(dd_w - fd_w) <= 1e-6 * float(np.abs(dv64 * w).sum())
