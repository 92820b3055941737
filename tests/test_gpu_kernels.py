"""GPU parity of the sparse kernels (SpMV, SpMV-transpose, blocked COO, Galerkin
product) against the CPU oracle, called through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import sparse as S  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, q1_problem, rel2, to_device_bsr  # noqa: E402


def _rand(nbr, nbc, br, bc, seed, **kw):
    rp, ci, v = synth.random_bsr(nbr, nbc, br, bc, seed, **kw)
    return S.Bsr(nbr, nbc, br, bc, rp.astype(np.int64), ci.astype(np.int64), v)


SHAPES = [(3, 3, 30), (3, 6, 6), (6, 3, 60), (6, 6, 30), (2, 5, 7), (1, 1, 9)]


@pytest.mark.parametrize("br,bc,per_row", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_spmv_f64_random(br, bc, per_row, nrhs):
    print(f"spmv f64 {br}x{bc} nrhs={nrhs}", flush=True)
    A = _rand(1037, 611, br, bc, seed=br * 7 + bc, max_per_row=per_row, empty_row_frac=0.05)
    H, keep = to_device_bsr(A)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (A.nbc * bc, nrhs))
    y0 = rng.uniform(-1, 1, (A.nbr * br, nrhs))
    want = S.spmv(A, x, 0.75, -0.5, y0)
    y = dev(y0)
    B.bsr_spmv(H, 0.75, dev(x), -0.5, y, nrhs=nrhs)
    assert rel2(y.cpu().numpy(), want) <= 1e-12
    # beta = 0 overwrites (NaN in y ignored)
    y = torch.full((A.nbr * br, nrhs), float("nan"), dtype=torch.float64, device="cuda")
    B.bsr_spmv(H, 1.0, dev(x), 0.0, y, nrhs=nrhs)
    assert rel2(y.cpu().numpy(), S.spmv(A, x)) <= 1e-12
    # transpose through the cached explicit transpose
    xt = rng.uniform(-1, 1, (A.nbr * br, nrhs))
    yt = torch.zeros((A.nbc * bc, nrhs), dtype=torch.float64, device="cuda")
    B.bsr_spmv_t(H, 1.0, dev(xt), 0.0, yt, nrhs=nrhs)
    assert rel2(yt.cpu().numpy(), S.spmv_t(A, xt)) <= 1e-12


def test_spmv_transpose_cache_follows_value_stamp():
    A = _rand(300, 200, 3, 6, seed=5, max_per_row=5)
    H, (rp, ci, v) = to_device_bsr(A)
    x = np.random.default_rng(2).uniform(-1, 1, A.nbr * 3)
    y = torch.zeros(A.nbc * 6, dtype=torch.float64, device="cuda")
    B.bsr_spmv_t(H, 1.0, dev(x), 0.0, y)
    assert rel2(y.cpu().numpy(), S.spmv_t(A, x)) <= 1e-12
    v.mul_(-2.0)
    B.bsr_mark_modified(H)
    B.bsr_spmv_t(H, 1.0, dev(x), 0.0, y)
    assert rel2(y.cpu().numpy(), -2.0 * S.spmv_t(A, x)) <= 1e-12


@pytest.mark.parametrize("br,bc", [(3, 3), (3, 6), (6, 6)])
def test_spmv_f32_and_bf16(br, bc):
    A = _rand(800, 500, br, bc, seed=11, max_per_row=20)
    x = np.random.default_rng(3).uniform(-1, 1, A.nbc * bc)
    want = S.spmv(A, x)
    H32, _ = to_device_bsr(A, B.F32)
    y = torch.zeros(A.nbr * br, dtype=torch.float32, device="cuda")
    B.bsr_spmv(H32, 1.0, dev(x, torch.float32), 0.0, y)
    assert rel2(y.cpu().numpy(), want) <= 2e-6
    if bc == 6:
        H16, _ = to_device_bsr(A, B.BF16)
        B.bsr_spmv(H16, 1.0, dev(x, torch.float32), 0.0, y)
        assert rel2(y.cpu().numpy(), want) <= 1e-2
        # exact w.r.t. the rounded values
        Ab = A.with_values(torch.as_tensor(A.val).to(torch.bfloat16).to(torch.float64).numpy())
        xf = torch.as_tensor(x).to(torch.float32).to(torch.float64).numpy()
        assert rel2(y.cpu().numpy(), S.spmv(Ab, xf)) <= 2e-6


def test_spmv_empty_and_errors():
    A = S.Bsr(5, 4, 3, 3, np.zeros(6, np.int64), np.zeros(0, np.int64), np.zeros((0, 3, 3)))
    H, _ = to_device_bsr(A)
    y = torch.ones(15, dtype=torch.float64, device="cuda")
    B.bsr_spmv(H, 1.0, torch.zeros(12, dtype=torch.float64, device="cuda"), 2.0, y)
    assert torch.all(y == 2.0)
    # vectors of the wrong element type are refused on the host, before any launch
    with pytest.raises(ValueError):
        B.bsr_spmv(H, 1.0, torch.zeros(12, device="cuda"), 0.0, torch.zeros(15, device="cuda"))
    with pytest.raises(ValueError):
        B.bsr_spmv(H, 1.0, torch.zeros(12, dtype=torch.float64, device="cuda"), 0.0, y, nrhs=9)
    # the library itself refuses the same calls (no launch)
    assert B._lib.bsr_spmv(H.h, 1.0, B._ptr(y), 0.0, B._ptr(y), B.F64, 9, None) == B.EINVAL
    assert B._lib.bsr_spmv(H.h, 1.0, B._ptr(y), 0.0, B._ptr(y), 7, 1, None) == B.EINVAL


def test_coo_plan_bit_exact_and_values():
    nbr, nbc = 257, 131
    i, j, v = synth.random_coo_stream(nbr, nbc, 3, 6, 20000, seed=4, neg_frac=0.1, dup_pool=3000)
    plan, H = B.coo_plan_create(nbr, nbc, 3, 6, i, j)
    rp, ci, perm, seg = S.coo_plan(nbr, nbc, i, j)
    dperm, dseg = plan.index_map()
    assert np.array_equal(dperm.cpu().numpy(), perm)
    assert np.array_equal(dseg.cpu().numpy(), seg)
    got_rp, got_ci, _ = H.arrays()
    assert np.array_equal(got_rp.cpu().numpy(), rp) and np.array_equal(got_ci.cpu().numpy(), ci)
    vals = dev(v)
    B.coo_assemble_blocked(plan, vals, B.INSERT, H)
    A = S.coo_assemble(nbr, nbc, i, j, v)
    got = from_device_bsr(H)
    assert np.array_equal(got.val, A.val)       # same summation order: identical bits
    B.coo_assemble_blocked(plan, vals, B.ADD, H)
    assert np.array_equal(from_device_bsr(H).val, 2 * A.val)
    with pytest.raises(B.BlkAmgError):
        B.coo_plan_create(nbr, nbc, 3, 6, np.array([nbr], np.int32), np.array([0], np.int32))


@pytest.mark.parametrize("br,bc", [(1, 1), (3, 3), (3, 6), (6, 6), (2, 2)])
@pytest.mark.parametrize("fp32", [False, True])
def test_coo_sum_every_block_shape(br, bc, fp32):
    # each block size has its own sum kernel (one or three components per thread,
    # or the generic loop): all keep the plan's stream order, so the bits match
    nbr, nbc = 301, 177
    i, j, v = synth.random_coo_stream(nbr, nbc, br, bc, 12000, seed=br * 10 + bc, neg_frac=0.1,
                                      dup_pool=2500)
    if fp32:
        v = v.astype(np.float32)
    plan, H = B.coo_plan_create(nbr, nbc, br, bc, i, j, val_dtype=B.F32 if fp32 else B.F64)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, H)
    want = S.coo_assemble(nbr, nbc, i, j, v.astype(np.float64)).val
    got = from_device_bsr(H).val
    if fp32:
        # the oracle sums in FP64; an FP32 sum of k terms is within k*eps of it
        scale = S.coo_assemble(nbr, nbc, i, j, np.abs(v).astype(np.float64)).val
        k = np.bincount(np.unique(i.astype(np.int64) * nbc + j, return_inverse=True)[1]).max()
        assert np.all(np.abs(got - want) <= (k + 1) * np.finfo(np.float32).eps * scale)
    else:
        assert np.array_equal(got, want)
    B.coo_assemble_blocked(plan, dev(v), B.ADD, H)
    got2 = from_device_bsr(H).val
    if fp32:
        assert np.all(np.abs(got2 - 2 * want) <= 2 * (k + 2) * np.finfo(np.float32).eps * scale)
    else:
        assert np.array_equal(got2, want + want)


@pytest.mark.parametrize("nbr,nbc,n,seed", [(257, 131, 20000, 4), (3000, 3000, 150000, 5), (1, 1, 50, 6)])
def test_coo_device_plan_bit_exact(nbr, nbc, n, seed):
    """The plan built on the device from device coordinates: the same index map, segments
    and pattern as the oracle's stable order by (row, column, position), bit for bit, and
    the same assembled values."""
    i, j, v = synth.random_coo_stream(nbr, nbc, 3, 3, n, seed=seed, neg_frac=0.1, dup_pool=max(n // 7, 1))
    print(f"device coo plan nbr={nbr} nbc={nbc} n={n}", flush=True)
    plan, H = B.coo_plan_create(nbr, nbc, 3, 3, dev(i), dev(j))
    rp, ci, perm, seg = S.coo_plan(nbr, nbc, i, j)
    dperm, dseg = plan.index_map()
    assert np.array_equal(dperm.cpu().numpy(), perm)
    assert np.array_equal(dseg.cpu().numpy(), seg)
    got_rp, got_ci, _ = H.arrays()
    assert np.array_equal(got_rp.cpu().numpy(), rp) and np.array_equal(got_ci.cpu().numpy(), ci)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, H)
    assert np.array_equal(from_device_bsr(H).val, S.coo_assemble(nbr, nbc, i, j, v).val)


def test_coo_device_plan_edge_cases():
    # empty stream, all entries ignored, one entry, out-of-range coordinate
    z = torch.zeros(0, dtype=torch.int32, device="cuda")
    plan, H = B.coo_plan_create(5, 5, 3, 3, z, z)
    assert H.info()["nnzb"] == 0 and plan.index_map()[1].cpu().tolist() == [0]
    neg = dev(np.array([-1, 2, -3], np.int32))
    plan, H = B.coo_plan_create(5, 5, 3, 3, neg, dev(np.array([1, -1, -1], np.int32)))
    assert H.info()["nnzb"] == 0 and H.arrays()[0].cpu().tolist() == [0] * 6
    plan, H = B.coo_plan_create(5, 4, 2, 2, dev(np.array([3], np.int32)), dev(np.array([2], np.int32)))
    rp, ci, _ = H.arrays()
    assert rp.cpu().tolist() == [0, 0, 0, 0, 1, 1] and ci.cpu().tolist() == [2]
    with pytest.raises(B.BlkAmgError) as e:
        B.coo_plan_create(5, 5, 3, 3, dev(np.array([0, 5], np.int32)), dev(np.array([0, 0], np.int32)))
    assert e.value.code == B.EINVAL and "entry 1" in str(e.value)


def test_coo_elasticity_stream_tiny_and_empty():
    m, i, j, v, A = q1_problem(8)
    plan, H = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, H)
    got = from_device_bsr(H)
    assert np.array_equal(got.rowptr, A.rowptr) and np.array_equal(got.colidx, A.colidx)
    assert got.nnzb == 13831
    assert np.array_equal(got.val, A.val)
    plan0, H0 = B.coo_plan_create(4, 4, 3, 3, np.array([-1, -1], np.int32), np.array([-1, 2], np.int32))
    B.coo_assemble_blocked(plan0, dev(np.zeros((2, 3, 3))), B.INSERT, H0)
    assert H0.info()["nnzb"] == 0


def test_ptap_random_against_oracle_and_stamp_gating():
    rp, ci, v = synth.random_spd_bsr(400, 3, seed=9, max_per_row=12)
    A = S.Bsr(400, 400, 3, 3, rp.astype(np.int64), ci.astype(np.int64), v)
    P = _rand(400, 57, 3, 6, seed=10, max_per_row=4)
    HA, _ = to_device_bsr(A)
    HP, (prp, pci, pv) = to_device_bsr(P)
    HC = B.ptap_symbolic(HA, HP)
    B.ptap_numeric(HA, HP, HC)
    want = S.ptap(A, P)
    got = from_device_bsr(HC)
    assert np.array_equal(got.rowptr, want.rowptr) and np.array_equal(got.colidx, want.colidx)
    assert rel2(got.val, want.val) <= 1e-12
    # new prolongator values: gated refresh of the cached transpose
    pv.mul_(0.5)
    B.bsr_mark_modified(HP)
    B.ptap_numeric(HA, HP, HC)
    assert rel2(from_device_bsr(HC).val, 0.25 * want.val) <= 1e-12
    # same values again: deterministic bits
    first = from_device_bsr(HC).val.copy()
    B.ptap_numeric(HA, HP, HC)
    assert np.array_equal(from_device_bsr(HC).val, first)
    # the plan's sizes: the A P pattern and the block products of both passes, counted
    # from the oracle's patterns
    pl = np.diff(P.rowptr)
    ap_len = np.array([len(np.unique(np.concatenate([P.colidx[P.rowptr[k]:P.rowptr[k + 1]]
                                                     for k in A.colidx[A.rowptr[r]:A.rowptr[r + 1]]])))
                       for r in range(A.nbr)])
    info = B.ptap_plan_info(HC)
    assert info["ap_nnzb"] == ap_len.sum() and not info["symmetric"]
    assert info["ap_pairs"] == pl[A.colidx].sum()
    assert info["c_pairs"] == (pl * ap_len).sum()
    with pytest.raises(B.BlkAmgError):
        B.ptap_plan_info(HA)


def test_ptap_coarse_6x6_and_f32():
    rp, ci, v = synth.random_spd_bsr(200, 6, seed=3, max_per_row=10)
    A = S.Bsr(200, 200, 6, 6, rp.astype(np.int64), ci.astype(np.int64), v)
    P = _rand(200, 31, 6, 6, seed=12, max_per_row=3)
    HA, _ = to_device_bsr(A)
    HP, _ = to_device_bsr(P)
    HC = B.ptap_symbolic(HA, HP)
    B.ptap_numeric(HA, HP, HC)
    want = S.ptap(A, P)
    assert rel2(from_device_bsr(HC).val, want.val) <= 1e-12
    HA32, _ = to_device_bsr(A, B.F32)
    HP32, _ = to_device_bsr(P, B.F32)
    HC32 = B.ptap_symbolic(HA32, HP32)
    B.ptap_numeric(HA32, HP32, HC32)
    assert rel2(from_device_bsr(HC32).val, want.val) <= 1e-5


def test_ptap_errors():
    A = _rand(10, 10, 3, 3, seed=1)
    P = _rand(11, 4, 3, 6, seed=2)
    HA, _ = to_device_bsr(A)
    HP, _ = to_device_bsr(P)
    with pytest.raises(B.BlkAmgError) as e:
        B.ptap_symbolic(HA, HP)
    assert e.value.code == B.EINVAL


def test_ptap_pair_lists_and_search_fallback_agree(monkeypatch):
    """The symbolic phase normally precomputes per-output contribution lists; with
    BLKAMG_PTAP_SEARCH=1 it keeps the searching kernels.  Both match the oracle."""
    m, i, j, v, A = q1_problem(7, 3)
    from oracle import solve
    H = solve.setup(A, m.coords, m.dirichlet, solve.Options(coarse_eq_limit=50))
    P = H.levels[0].P
    HA, _ = to_device_bsr(A)
    HP, _ = to_device_bsr(P)
    want = S.ptap(A, P)
    C1 = B.ptap_symbolic(HA, HP)
    B.ptap_numeric(HA, HP, C1)
    monkeypatch.setenv("BLKAMG_PTAP_SEARCH", "1")
    C2 = B.ptap_symbolic(HA, HP)
    B.ptap_numeric(HA, HP, C2)
    g1, g2 = from_device_bsr(C1), from_device_bsr(C2)
    assert rel2(g1.val, want.val) <= 1e-12 and rel2(g2.val, want.val) <= 1e-12
    assert np.array_equal(g1.val, g2.val)   # same summation order in both kernels


@pytest.mark.parametrize("bs", [3, 6])
def test_ptap_symmetric_mode(bs):
    """BLKAMG_PTAP_SYMMETRIC computes the upper blocks and mirrors them: same values
    as the oracle within 1e-12, and the result is exactly symmetric."""
    rp, ci, v = synth.random_spd_bsr(300, bs, seed=21, max_per_row=10)
    A = S.Bsr(300, 300, bs, bs, rp.astype(np.int64), ci.astype(np.int64), v)
    P = _rand(300, 41, bs, 6, seed=22, max_per_row=4)
    HA, _ = to_device_bsr(A)
    HP, _ = to_device_bsr(P)
    HC = B.ptap_symbolic_ex(HA, HP, B.PTAP_SYMMETRIC)
    B.ptap_numeric(HA, HP, HC)
    want = S.ptap(A, P)
    got = from_device_bsr(HC)
    assert np.array_equal(got.rowptr, want.rowptr) and np.array_equal(got.colidx, want.colidx)
    assert rel2(got.val, want.val) <= 1e-12
    rows = got.block_rows()
    pos = {(int(r), int(c)): t for t, (r, c) in enumerate(zip(rows, got.colidx))}
    for t, (r, c) in enumerate(zip(rows, got.colidx)):
        if r != c:   # mirrored: exact
            assert np.array_equal(got.val[t], got.val[pos[(int(c), int(r))]].T)
        else:        # computed directly: symmetric to rounding
            assert np.abs(got.val[t] - got.val[t].T).max() <= 1e-13 * np.abs(got.val[t]).max()
    with pytest.raises(B.BlkAmgError):
        B.ptap_symbolic_ex(HA, HP, 8)


@pytest.mark.parametrize("bs", [3, 6])
def test_ptap_lane_mappings_agree(bs, monkeypatch):
    """One or three lanes per output block (each lane owning a share of its columns),
    LDS-staged or global-memory workgroups: every mapping adds the same products in
    the same order, so all give identical bits, within 1e-12 (FP64) / 1e-5 (FP32) of
    the oracle."""
    rp, ci, v = synth.random_spd_bsr(300, bs, seed=31, max_per_row=14)
    A = S.Bsr(300, 300, bs, bs, rp.astype(np.int64), ci.astype(np.int64), v)
    P = _rand(300, 41, bs, 6, seed=32, max_per_row=5)
    want = S.ptap(A, P)
    for dt, tol in ((B.F64, 1e-12), (B.F32, 1e-5)):
        HA, _ = to_device_bsr(A, dt)
        HP, _ = to_device_bsr(P, dt)
        ref = None
        for tune in ("ap_sort,ap_nl1,c_nl1", "ap_sort,ap_nl3,c_nl3", "ap_sort,ap_nl3,c_nl1",
                     "ap_sort,ap_nl1,c_nl3,nostage", "ap_sort,ap_nl3,c_nl3,nostage",
                     "ap_sort,ap_nl3,c_nl1,ap_xcd,c_xcd", "ap_sort,ap_nl3,c_nl3,ap_xcd=0,c_xcd=0",
                     "ap_sort,ap_nl3,c_nl3,ap_xcd=3,c_xcd=5"):
            monkeypatch.setenv("BLKAMG_PTAP_TUNE", tune)
            HC = B.ptap_symbolic_ex(HA, HP, B.PTAP_SYMMETRIC)
            B.ptap_numeric(HA, HP, HC)
            got = from_device_bsr(HC)
            assert rel2(got.val, want.val) <= tol, tune
            if ref is None:
                ref = got.val.copy()
            else:
                assert np.array_equal(got.val, ref), tune


@pytest.mark.parametrize("bs", [3, 6])
def test_spmv_sym_is_the_symmetric_completion(bs):
    """bsr_spmv_sym applies S (A's diagonal and upper blocks, lower blocks as transposed
    mirrors): against the oracle's S on a symmetric pattern with unrelated values, and
    equal to bsr_spmv on a symmetric matrix up to the grouping of the row sums (the
    symmetric reads use their own lane shape), F64 and F32."""
    print(f"spmv_sym bs={bs}", flush=True)
    rp, ci, v = synth.random_spd_bsr(2311, bs, seed=bs, max_per_row=9)
    A = S.Bsr(2311, 2311, bs, bs, rp.astype(np.int64), ci.astype(np.int64), v)
    W = A.with_values(np.random.default_rng(bs).uniform(-1, 1, A.val.shape))
    x = np.random.default_rng(2).uniform(-1, 1, A.nbr * bs)
    y0 = np.random.default_rng(3).uniform(-1, 1, A.nbr * bs)
    HW, _ = to_device_bsr(W)
    y = dev(y0)
    B.bsr_spmv_sym(HW, 0.5, dev(x), -2.0, y)
    assert rel2(y.cpu().numpy(), S.spmv(S.symmetric_completion(W), x, 0.5, -2.0, y0)) <= 1e-13
    for dt, tdt in ((B.F64, torch.float64), (B.F32, torch.float32)):
        HA, _ = to_device_bsr(A, dt)
        xs = dev(x, tdt)
        y1 = torch.zeros(A.nbr * bs, dtype=tdt, device="cuda")
        y2 = torch.zeros_like(y1)
        B.bsr_spmv(HA, 1.0, xs, 0.0, y1)
        B.bsr_spmv_sym(HA, 1.0, xs, 0.0, y2)
        assert rel2(y2.double().cpu().numpy(), y1.double().cpu().numpy()) <= (1e-15 if dt == B.F64 else 1e-7), dt


def test_spmv_sym_on_the_elasticity_operator_and_refusals():
    """The assembled Q1 operator is symmetric bit for bit, so the symmetric reads apply A
    itself (equal to the full reads up to the grouping of the row sums, against the
    oracle at 1e-14); rectangular blocks and unsymmetric patterns are refused."""
    m, i, j, v, A = q1_problem(14, mat_seed=3)
    HA, _ = to_device_bsr(A)
    x = dev(np.random.default_rng(7).uniform(-1, 1, A.nbr * 3))
    y1 = torch.zeros(A.nbr * 3, dtype=torch.float64, device="cuda")
    y2 = torch.zeros_like(y1)
    B.bsr_spmv(HA, 1.0, x, 0.0, y1)
    B.bsr_spmv_sym(HA, 1.0, x, 0.0, y2)
    assert rel2(y2.cpu().numpy(), y1.cpu().numpy()) <= 1e-15
    assert rel2(y2.cpu().numpy(), S.spmv(A, x.cpu().numpy())) <= 1e-14
    R = _rand(40, 30, 3, 6, seed=1)
    HR, _ = to_device_bsr(R)
    with pytest.raises(B.BlkAmgError) as e:
        B.bsr_spmv_sym(HR, 1.0, dev(np.zeros(180)), 0.0, torch.zeros(120, dtype=torch.float64, device="cuda"))
    assert e.value.code == B.EINVAL
    U = S.Bsr(3, 3, 3, 3, np.array([0, 1, 3, 4]), np.array([0, 0, 1, 2]), np.ones((4, 3, 3)))
    HU, _ = to_device_bsr(U)
    with pytest.raises(B.BlkAmgError):
        B.bsr_spmv_sym(HU, 1.0, dev(np.zeros(9)), 0.0, torch.zeros(9, dtype=torch.float64, device="cuda"))


def test_spmv_sym_follows_the_values():
    """The symmetric reads see the current values: after the library changes them (COO
    assembly) and after the caller writes them (declared with bsr_mark_modified); a
    pattern whose mirror search fails on a row listed out of order is refused."""
    m, i, j, v, A = q1_problem(6, mat_seed=5)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    x = dev(np.random.default_rng(11).uniform(-1, 1, A.nbr * 3))
    y = torch.zeros(A.nbr * 3, dtype=torch.float64, device="cuda")
    for scale in (1.0, 2.5):
        B.coo_assemble_blocked(plan, dev(v * scale), B.INSERT, HA)
        B.bsr_spmv_sym(HA, 1.0, x, 0.0, y)
        assert rel2(y.cpu().numpy(), scale * S.spmv(A, x.cpu().numpy())) <= 1e-14, scale
    # a matrix over caller arrays, its values then changed by the caller
    rpt = torch.as_tensor(A.rowptr.astype(np.int32), device="cuda")
    cit = torch.as_tensor(A.colidx.astype(np.int32), device="cuda")
    vt = torch.as_tensor(A.val.reshape(-1).copy(), device="cuda")
    HB = B.bsr_create(A.nbr, A.nbc, 3, 3, rpt, cit, vt)
    B.bsr_spmv_sym(HB, 1.0, x, 0.0, y)
    assert rel2(y.cpu().numpy(), S.spmv(A, x.cpu().numpy())) <= 1e-14
    vt.mul_(-3.0)
    B.bsr_mark_modified(HB)
    B.bsr_spmv_sym(HB, 1.0, x, 0.0, y)
    assert rel2(y.cpu().numpy(), -3.0 * S.spmv(A, x.cpu().numpy())) <= 1e-14
    # symmetric pattern, but row 1 lists its columns out of order
    rp = torch.tensor([0, 2, 4, 6], dtype=torch.int32, device="cuda")
    ci = torch.tensor([0, 1, 1, 0, 1, 2], dtype=torch.int32, device="cuda")
    vv = torch.ones(6 * 9, dtype=torch.float64, device="cuda")
    HU = B.bsr_create(3, 3, 3, 3, rp, ci, vv)
    with pytest.raises(B.BlkAmgError):
        B.bsr_spmv_sym(HU, 1.0, dev(np.zeros(9)), 0.0, torch.zeros(9, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("case", ["q1_sym", "q1_full", "rand6_sym", "rand3_empty_rows", "f32_sym", "c_sort_nostage",
                                  "q2_long_rows_sym", "q2_long_rows_full"])
def test_ptap_device_symbolic_equals_host_build(case, monkeypatch):
    """The symbolic phase built on the device (default) and on the host
    (PTAP_HOST_SYMBOLIC) give the same coarse pattern and, through the same contribution
    order, the same numeric bits; both match the oracle's P^T A P."""
    print(f"device symbolic case={case}", flush=True)
    dt, flags = B.F64, B.PTAP_SYMMETRIC
    if case.startswith("q1") or case == "f32_sym" or case == "c_sort_nostage":
        m, i, j, v, A = q1_problem(9, 3)
        from oracle import solve
        P = solve.setup(A, m.coords, m.dirichlet, solve.Options(coarse_eq_limit=50)).levels[0].P
        if case == "q1_full":
            flags = 0
        if case == "f32_sym":
            dt = B.F32
        if case == "c_sort_nostage":
            monkeypatch.setenv("BLKAMG_PTAP_TUNE", "ap_sort,c_sort,nostage")
    elif case.startswith("q2"):
        # triquadratic elements at 5^3: coarse rows with up to 4,913 contributions, beyond
        # the LDS sort (4096), so they take the device-memory sort
        m, i, j, v, A = q1_problem(5, 3, order=2)
        from oracle import solve
        P = solve.setup(A, m.coords, m.dirichlet).levels[0].P
        if case.endswith("full"):
            flags = 0
    elif case == "rand6_sym":
        rp, ci, vv = synth.random_spd_bsr(500, 6, seed=41, max_per_row=12)
        A = S.Bsr(500, 500, 6, 6, rp.astype(np.int64), ci.astype(np.int64), vv)
        P = _rand(500, 63, 6, 6, seed=42, max_per_row=4)
    else:
        A = _rand(600, 600, 3, 3, seed=43, max_per_row=20, empty_row_frac=0.1)
        P = _rand(600, 70, 3, 6, seed=44, max_per_row=5, empty_row_frac=0.2)
        flags = 0
    HA, _ = to_device_bsr(A, dt)
    HP, _ = to_device_bsr(P, dt)
    Cd = B.ptap_symbolic_ex(HA, HP, flags)
    Ch = B.ptap_symbolic_ex(HA, HP, flags | B.PTAP_HOST_SYMBOLIC)
    B.ptap_numeric(HA, HP, Cd)
    B.ptap_numeric(HA, HP, Ch)
    gd, gh = from_device_bsr(Cd), from_device_bsr(Ch)
    want = S.ptap(A, P)
    assert np.array_equal(gd.rowptr, want.rowptr) and np.array_equal(gd.colidx, want.colidx)
    assert np.array_equal(gd.rowptr, gh.rowptr) and np.array_equal(gd.colidx, gh.colidx)
    assert np.array_equal(gd.val, gh.val)
    assert rel2(gd.val, want.val) <= (1e-12 if dt == B.F64 else 1e-5)
