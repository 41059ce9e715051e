"""GPU format construction (COO -> CRS, CRS -> JDS, JDS -> blocked JDS, transpose)
against the oracle: integer and index work must be bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import gpu_csr, rand_coo, to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")


def test_csr_from_coo_shuffled_duplicates():
    rng = np.random.default_rng(1)
    n_rows, n_cols, k = 3000, 2500, 60000
    row = rng.integers(0, n_rows, k).astype(np.int32)
    col = rng.integers(0, n_cols, k).astype(np.int32)
    row[:500] = 7                      # a long row and many duplicates
    col[:500] = rng.integers(0, 40, 500)
    val = rng.standard_normal(k)
    val[::13] = 0.0
    A = gpu_csr(sp, row, col, val, n_rows, n_cols)
    R = oracle.csr_from_coo(n_rows, n_cols, row, col, val)
    assert np.array_equal(to_np(A.row_ptr), R.row_ptr)
    assert np.array_equal(to_np(A.col_idx), R.col)
    assert np.array_equal(to_np(A.val), R.val)      # sums in input order: bit-exact
    assert sp.spmv_csr_validate(A)


def test_csr_from_coo_float32_and_empty_and_errors():
    r, c, v, nr, nc, _ = rand_coo(2, 700, 900, 0.02, empty_rows=0.3)
    order = np.random.default_rng(3).permutation(len(r))
    A = gpu_csr(sp, r[order], c[order], v[order], nr, nc, torch.float32)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    assert np.array_equal(to_np(A.row_ptr), R.row_ptr)
    assert np.array_equal(to_np(A.col_idx), R.col)
    assert np.array_equal(to_np(A.val), R.val.astype(np.float32))
    E = sp.csr_from_coo(5, 5, to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0, np.int32)),
                        to_dev(np.zeros(0)))
    assert E.nnz == 0 and to_np(E.row_ptr).tolist() == [0] * 6
    with pytest.raises(sp.SpmvError):
        sp.csr_from_coo(3, 3, to_dev(np.array([0, 3], np.int32)), to_dev(np.array([0, 0], np.int32)),
                        to_dev(np.ones(2)))


def test_validate_detects_bad_structure():
    r, c, v, nr, nc, _ = rand_coo(4, 100, 100, 0.05)
    A = gpu_csr(sp, r, c, v, nr, nc)
    assert sp.spmv_csr_validate(A)
    bad = A.col_idx.clone()
    bad[3] = nc + 5
    assert not sp.spmv_csr_validate(A.__class__(nr, nc, A.row_ptr, bad, A.val))
    rp = A.row_ptr.clone()
    rp[10] = rp[11] + 5                      # row_ptr decreases at row 10
    assert not sp.spmv_csr_validate(A.__class__(nr, nc, rp, A.col_idx, A.val))


def check_jds(J, R):
    assert np.array_equal(to_np(J.perm), R.perm)
    assert np.array_equal(to_np(J.iperm), R.iperm)
    assert np.array_equal(to_np(J.jd_ptr), R.jd_ptr)
    assert np.array_equal(J.h_jd_ptr, R.jd_ptr)
    assert np.array_equal(to_np(J.jd_col), R.jd_col)
    assert np.array_equal(to_np(J.jd_val).astype(np.float64), R.jd_val)


@pytest.mark.parametrize("symperm", [False, True])
def test_jds_from_csr_bit_exact(symperm):
    r, c, v, nr, nc, _ = rand_coo(5, 5000, 5000, 0.002, empty_rows=0.2, long_rows=5, long_len=700)
    A = gpu_csr(sp, r, c, v, nr, nc)
    Rc = oracle.csr_from_coo(nr, nc, r, c, v)
    J = sp.jds_from_csr(A, symperm=symperm)
    check_jds(J, oracle.jds_from_csr(Rc, symperm=symperm))
    B = sp.jds_to_csr(J)                        # exact inverse
    assert np.array_equal(to_np(B.row_ptr), Rc.row_ptr)
    assert np.array_equal(to_np(B.col_idx), Rc.col)
    assert np.array_equal(to_np(B.val), Rc.val)


def test_jds_laplacian_jd_ptr():
    r, c, v, n, _ = synth.laplacian3d(20)
    J = sp.jds_from_csr(gpu_csr(sp, r, c, v, n, n))
    assert J.h_jd_ptr.tolist() == [0, 8000, 16000, 24000, 32000, 39992, 47768, 53600]


@pytest.mark.parametrize("C", [64, 128, 512])
@pytest.mark.parametrize("sojds", [False, True])
def test_blocked_from_jds_bit_exact(C, sojds):
    r, c, v, nr, nc, _ = rand_coo(6, 3000, 3000, 0.003, empty_rows=0.1, long_rows=3, long_len=300)
    Rc = oracle.csr_from_coo(nr, nc, r, c, v)
    Rb = oracle.blocked_from_jds(oracle.jds_from_csr(Rc), C, sojds=sojds)
    J = sp.jds_from_csr(gpu_csr(sp, r, c, v, nr, nc))
    B = sp.jds_blocked_from_jds(J, C, sojds=sojds)
    assert np.array_equal(to_np(B.slice_ptr), Rb.slice_ptr)
    assert np.array_equal(to_np(B.slice_nd), Rb.slice_nd)
    assert np.array_equal(B.h_slice_nd, Rb.slice_nd)
    assert np.array_equal(to_np(B.bl_col), Rb.bl_col)
    assert np.array_equal(to_np(B.bl_val), Rb.bl_val)


@pytest.mark.parametrize("shuffle", [False, True])
def test_sojds_long_and_unsorted_rows_bit_exact(shuffle):
    """SOJDS on rows of up to 2,500 entries (the logarithmic search of sorted
    rows) and, with `shuffle`, on a CRS whose rows are not in column order
    (the direct search): bit-exact against the oracle's greedy rule."""
    r, c, v, nr, nc, rng = rand_coo(8, 1500, 4000, 0.004, empty_rows=0.1, long_rows=40, long_len=2500)
    Rc = oracle.csr_from_coo(nr, nc, r, c, v)
    if shuffle:
        col, val = Rc.col.copy(), Rc.val.copy()
        for i in rng.choice(nr, nr // 3, replace=False):
            a, b = Rc.row_ptr[i], Rc.row_ptr[i + 1]
            p = rng.permutation(b - a)
            col[a:b], val[a:b] = col[a:b][p], val[a:b][p]
        Rc = oracle.CSR(nr, nc, Rc.row_ptr, col, val)
    A = sp.CSR(nr, nc, to_dev(Rc.row_ptr), to_dev(Rc.col), to_dev(Rc.val))
    for C in (64, 256):
        Rb = oracle.blocked_from_jds(oracle.jds_from_csr(Rc), C, sojds=True)
        B = sp.jds_blocked_from_jds(sp.jds_from_csr(A), C, sojds=True)
        assert np.array_equal(to_np(B.bl_col), Rb.bl_col), C
        assert np.array_equal(to_np(B.bl_val), Rb.bl_val), C


def test_sojds_rows_past_the_lds_capacity_bit_exact():
    """Slices whose first row has more than 4,096 entries take the serial
    builder, the others the wavefront builder: both bit-exact against the
    oracle's greedy rule, in one storage."""
    r, c, v, nr, nc, rng = rand_coo(9, 1200, 6000, 0.003, empty_rows=0.1, long_rows=5, long_len=5000)
    Rc = oracle.csr_from_coo(nr, nc, r, c, v)
    A = sp.CSR(nr, nc, to_dev(Rc.row_ptr), to_dev(Rc.col), to_dev(Rc.val))
    Rb = oracle.blocked_from_jds(oracle.jds_from_csr(Rc), 64, sojds=True)
    B = sp.jds_blocked_from_jds(sp.jds_from_csr(A), 64, sojds=True)
    assert np.array_equal(to_np(B.bl_col), Rb.bl_col)
    assert np.array_equal(to_np(B.bl_val), Rb.bl_val)


@pytest.mark.parametrize("C,sigma", [(64, 64), (64, 256), (128, 384), (64, 1 << 20)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32, torch.int32])
def test_windowed_blocked_bit_exact(C, sigma, dt):
    """The windowed RBJDS builder against the oracle's: perm, slice pointers
    and depths, and every padded slot, bit for bit (empty rows, rows of
    5,000 entries, a ragged last slice)."""
    r, c, v, nr, nc, rng = rand_coo(95, 5003, 6000, 0.002, empty_rows=0.2, long_rows=3, long_len=5000)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    Bo = oracle.blocked_windowed(R, C, sigma)
    A = sp.csr_from_coo(nr, nc, to_dev(r), to_dev(c), to_dev(v))
    if dt == torch.int32:
        # int32 payload: each entry's CRS position, laid out by the oracle
        A = A.with_values(torch.arange(A.nnz, dtype=torch.int32, device="cuda"))
        Bp = oracle.blocked_windowed(oracle.CSR(nr, nc, R.row_ptr, R.col, np.arange(R.nnz, dtype=np.float64)), C,
                                     sigma)
        want_val = Bp.bl_val.astype(np.int64)
    elif dt == torch.float32:
        A = A.with_values(sp.spmv_convert_values(A.val, torch.float32))
        want_val = oracle.round_f32(Bo.bl_val)
    else:
        want_val = Bo.bl_val
    B = sp.jds_blocked_windowed_from_csr(A, C, sigma)
    assert np.array_equal(to_np(B.perm), Bo.perm)
    assert np.array_equal(to_np(B.slice_ptr), Bo.slice_ptr)
    assert np.array_equal(B.h_slice_nd, Bo.slice_nd) and np.array_equal(to_np(B.slice_nd), Bo.slice_nd)
    assert np.array_equal(to_np(B.bl_col), Bo.bl_col)
    got = to_np(B.bl_val)
    assert np.array_equal(got.astype(np.int64) if dt == torch.int32 else got, want_val)


def test_windowed_blocked_rejects_and_empty():
    A = sp.csr_from_coo(10, 10, to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0, np.int32)), to_dev(np.zeros(0)))
    B = sp.jds_blocked_windowed_from_csr(A, 64, 64)
    assert B.padded == 0 and B.h_slice_nd.tolist() == [0]
    y = sp.spmv_jds_blocked_tiled(B, to_dev(np.ones(10)), to_dev(np.full(10, 3.0)), 1.0, 0.5)
    assert to_np(y).tolist() == [1.5] * 10
    from paper_0910_4836_amd import _lib
    lib = _lib.load()
    st = lib.spmv_jds_blocked_windowed_from_csr(10, 0, None, None, None, 0, 64, 96, None, None, None, None, None, 0,
                                                None, None, None, 0, None)
    assert st == 1 and b"multiple of C" in lib.spmv_last_error()


def test_transpose_bit_exact():
    r, c, v, nr, nc, _ = rand_coo(7, 2000, 1500, 0.004, empty_rows=0.1)
    Rc = oracle.csr_from_coo(nr, nc, r, c, v)
    rowT, colT, tmap = oracle.transpose(Rc)
    A = gpu_csr(sp, r, c, v, nr, nc)
    gr, gc, gt = sp.spmv_transpose_csr(A)
    assert np.array_equal(to_np(gr), rowT)
    assert np.array_equal(to_np(gc), colT)
    assert np.array_equal(to_np(gt).astype(np.int64), tmap)


def test_convert_values_rounding():
    rng = np.random.default_rng(8)
    v = np.concatenate([rng.standard_normal(100000), rng.standard_normal(1000) * 1e-39,
                        rng.standard_normal(1000) * 3e38,
                        [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -40, 2.0 ** -134, 511 * 2.0 ** 119,
                         0.0, -0.0, np.inf, -np.inf]])
    t = to_dev(v)
    b = sp.spmv_convert_values(t, torch.bfloat16)
    assert np.array_equal(to_np(b.view(torch.int16)).view(np.uint16), oracle.round_bf16_bits(v))
    f = sp.spmv_convert_values(t, torch.float32)
    assert np.array_equal(to_np(f), oracle.round_f32(v))
    back = sp.spmv_convert_values(b, torch.float64)
    assert np.array_equal(to_np(back), oracle.bf16_bits_to_f64(oracle.round_bf16_bits(v)))


def test_permute_and_gather():
    rng = np.random.default_rng(9)
    n = 10000
    perm = rng.permutation(n).astype(np.int32)
    v = rng.standard_normal(n)
    p, t = to_dev(perm), to_dev(v)
    assert np.array_equal(to_np(sp.spmv_permute_vec(p, t)), v[perm])
    out = np.empty(n)
    out[perm] = v
    assert np.array_equal(to_np(sp.spmv_permute_vec(p, t, inverse=True)), out)
    idx = rng.integers(0, n, 3000).astype(np.int32)
    assert np.array_equal(to_np(sp.spmv_gather_values(to_dev(idx), t)), v[idx])
    iv = rng.integers(-2 ** 31, 2 ** 31 - 1, n).astype(np.int32)
    assert np.array_equal(to_np(sp.spmv_gather_values(to_dev(idx), to_dev(iv))), iv[idx])


def test_bandwidth_and_gather_probes():
    """The probes compute what they read: integer-valued data, exact sums."""
    n = 1 << 20
    b = torch.arange(n, dtype=torch.float64, device="cuda") % 7
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    sp.spmv_stream_triad(a, b, c, 0.5)
    assert torch.equal(a, b + 1.0)
    sp.spmv_stream_copy(a, c)
    assert torch.equal(a, c)
    part = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    sp.spmv_stream_read(b, part)
    assert part.sum().item() == b.sum().item()
    x = (torch.arange(5000, dtype=torch.float64, device="cuda") % 13) - 6
    idx = torch.from_numpy(np.random.default_rng(3).integers(0, 5000, 300001).astype(np.int32)).cuda()
    part.zero_()
    sp.spmv_gather_probe(idx, x, part)
    assert part.sum().item() == x[idx.long()].sum().item()


@pytest.mark.parametrize("n", [1, 255, 2048 * 8 + 77, 600_001])
def test_stride_probe(n):
    """The access-pattern probe sums what its index stream names: small
    integers, so every order of the sum is exact."""
    rng = np.random.default_rng(n)
    av = rng.integers(-4, 5, n).astype(np.float64)
    bv = rng.integers(-4, 5, 64 * n + 1).astype(np.float64)
    a, b = to_dev(av), to_dev(bv)
    part = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    for k in (1, 3, 64):
        j = np.arange(n) * k
        for scp in (False, True):
            part.zero_()
            sp.spmv_stride_probe(n, b, part, a=a if scp else None, k=k)
            want = (av * bv[j]).sum() if scp else bv[j].sum()
            assert part.sum().item() == want, (k, scp)
    streams = {"IS": synth.index_stream("IS", n, 5, rng), "IR": synth.index_stream("IR", n, 7, rng),
               "GAUSS": synth.index_stream("GAUSS", n, 3, rng, 40.0)}
    for kind, ind in streams.items():
        ind = np.minimum(ind, len(bv) - 1)
        it = to_dev(ind.astype(np.int32))
        for scp in (False, True):
            part.zero_()
            sp.spmv_stride_probe(n, b, part, a=a if scp else None, ind=it, ind_max=int(ind.max()))
            want = (av * bv[ind]).sum() if scp else bv[ind].sum()
            assert part.sum().item() == want, (kind, scp)


def test_stride_probe_rejects():
    b = torch.ones(100, dtype=torch.float64, device="cuda")
    part = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    sp.spmv_stride_probe(0, b, part)                                  # empty: nothing to do
    with pytest.raises(ValueError):
        sp.spmv_stride_probe(51, b, part, k=2)                        # index 100 is past b
    with pytest.raises(sp.SpmvError):
        sp.spmv_stride_probe(100, b, part, k=0)
    with pytest.raises(sp.SpmvError):
        sp.spmv_stride_probe(100, b, part[:0])                        # no room for the partial sums
