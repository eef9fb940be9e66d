"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every input comes from the seeded generators; every expected value from the
oracle. Tolerances (normwise relative error):
  * FP32 vectors/factors vs the oracle on the same FP32 values:      1e-5
  * BF16 vectors/factors vs the oracle on the BF16-rounded values:   1e-5
  * BF16 vectors/factors vs the oracle on the original FP64 values:  2e-2
  * SYPRD: |s - s_ref| <= 1e-5 * sum of |terms| (the scalar can cancel)
  * integer results (expansion counts, pattern histogram): bit-exact
FP32 atomics make the GPU's summation order vary between runs, so several
last-bit results are correct; the tolerance covers them.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_2406_09266_amd as systec
from paper_2406_09266_amd import synth

from gpu_util import assert_elementwise, dev, f32, rel_err

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_BF16_E2E = 2e-2


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _bf16_round(a):
    return oracle.round_bf16(np.asarray(a, dtype=np.float32))


def _ssymv_case(m, xdtype="f32"):
    import torch
    n = m["n"]
    val32 = f32(m["val"])
    x32 = f32(m["x"])
    rp, col = dev(m["rowptr"]), dev(m["col"])
    val = dev(m["val"].astype(np.float32))
    if xdtype == "f32":
        x = dev(m["x"].astype(np.float32))
        x_ref = x32
    else:
        x = systec.quantize_bf16(dev(m["x"].astype(np.float32)))
        x_ref = _bf16_round(m["x"])
    y = systec.ssymv(rp, col, val, x).cpu().numpy()
    want, counts = oracle.ssymv(n, m["rowptr"], m["col"], val32, x_ref)
    return y, want, counts


# ------------------------------------------------------------------- SSYMV --

SSYMV_CASES = {
    "small_n2000": lambda: synth.workload("ssymv_small"),
    "uniform_n5000_ragged": lambda: synth.ssymv_uniform(5003, 9, seed=11),
    "rmat_scale14_hubs": lambda: synth.ssymv_rmat(scale=14, batch=1 << 16, seed=12),
    "rmat_scale16_relabel": lambda: synth.ssymv_rmat(scale=16, batch=1 << 18, seed=13,
                                                     relabel=True),
    "diagonal_only": lambda: synth.ssymv_uniform(3000, 0, seed=14),
    "random_degree": lambda: synth.ssymv_random_degree(20000, 12, seed=15),
}


@pytest.mark.parametrize("case", sorted(SSYMV_CASES))
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_ssymv_matches_oracle(case, xdtype):
    m = SSYMV_CASES[case]()
    print(f"ssymv case={case} x={xdtype} n={m['n']} nnz={m['col'].size}", flush=True)
    y, want, _ = _ssymv_case(m, xdtype)
    assert rel_err(y, want) <= TOL32
    if xdtype == "bf16":
        full, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], m["val"], m["x"])
        assert rel_err(y, full) <= TOL_BF16_E2E


# matrices of at least 2^18 stored entries, where the one-shot SSYMV bins
# the column side by ranges of 16,384 columns (several buckets, a ragged
# last bucket, hub rows, rows without entries)
SSYMV_BUCKETED_CASES = {
    "rmat_scale18": lambda: synth.ssymv_rmat(scale=18, batch=1 << 21, seed=31),
    "uniform_n70001": lambda: synth.ssymv_uniform(70001, 9, seed=32),
    "random_degree_n150000": lambda: synth.ssymv_random_degree(150000, 6, seed=33),
}


@pytest.mark.parametrize("case", sorted(SSYMV_BUCKETED_CASES))
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_ssymv_bucketed_matches_oracle(case, xdtype):
    m = SSYMV_BUCKETED_CASES[case]()
    assert m["col"].size >= 1 << 18
    print(f"ssymv bucketed case={case} x={xdtype} n={m['n']} nnz={m['col'].size}", flush=True)
    y, want, _ = _ssymv_case(m, xdtype)
    x_ref = f32(m["x"]) if xdtype == "f32" else _bf16_round(m["x"])
    scale, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], np.abs(f32(m["val"])), np.abs(x_ref))
    assert_elementwise(y, want, scale, TOL32, f"ssymv bucketed {case}")
    assert rel_err(y, want) <= TOL32


def test_ssymv_bucketed_one_long_row():
    # row 0 holds every column of a 300,000-column matrix: one row across
    # every bucket, every other row empty
    n = 300000
    rowptr = np.full(n + 1, n, dtype=np.int32)
    rowptr[0] = 0
    m = {"n": n, "rowptr": rowptr, "col": np.arange(n, dtype=np.int32),
         "val": synth.dense_uniform(n, seed=5), "x": synth.dense_uniform(n, seed=6)}
    y, want, _ = _ssymv_case(m)
    scale, _ = oracle.ssymv(n, m["rowptr"], m["col"], np.abs(f32(m["val"])), np.abs(f32(m["x"])))
    assert_elementwise(y, want, scale, TOL32, "ssymv bucketed long row")


def test_ssymv_empty_and_single():
    import torch
    n = 37
    rp = dev(np.zeros(n + 1, dtype=np.int32))
    empty_i = torch.empty(0, dtype=torch.int32, device="cuda")
    empty_f = torch.empty(0, dtype=torch.float32, device="cuda")
    x = dev(synth.dense_uniform(n, seed=1).astype(np.float32))
    y = systec.ssymv(rp, empty_i, empty_f, x, out=torch.full((n,), 7.0, device="cuda"))
    assert torch.count_nonzero(y).item() == 0
    # n = 1, one diagonal entry
    y1 = systec.ssymv(dev(np.array([0, 1], np.int32)), dev(np.array([0], np.int32)),
                      dev(np.array([2.5], np.float32)), dev(np.array([-3.0], np.float32)))
    assert y1.item() == -7.5


def test_ssymv_one_long_row_spanning_tiles():
    # row 0 holds every column: one segment across many wavefront tiles
    n = 20000
    rowptr = np.concatenate([[0], np.full(n, n, dtype=np.int64)]).astype(np.int32)
    rowptr[1:] = n
    m = {"n": n, "rowptr": rowptr, "col": np.arange(n, dtype=np.int32),
         "val": synth.dense_uniform(n, seed=3), "x": synth.dense_uniform(n, seed=4)}
    y, want, _ = _ssymv_case(m)
    assert rel_err(y, want) <= TOL32


def test_syprd_matches_oracle():
    for m in (synth.workload("ssymv_small"), synth.ssymv_rmat(scale=14, batch=1 << 16, seed=21)):
        val32, x32 = f32(m["val"]), f32(m["x"])
        rp, col = dev(m["rowptr"]), dev(m["col"])
        val, x = dev(m["val"].astype(np.float32)), dev(m["x"].astype(np.float32))
        s = systec.syprd(rp, col, val, x).item()
        want, scale, _ = oracle.syprd(m["n"], m["rowptr"], m["col"], val32, x32)
        assert abs(s - want) <= TOL32 * scale
        xb = systec.quantize_bf16(x)
        sb = systec.syprd(rp, col, val, xb).item()
        wantb, scaleb, _ = oracle.syprd(m["n"], m["rowptr"], m["col"], val32, _bf16_round(m["x"]))
        assert abs(sb - wantb) <= TOL32 * scaleb


def test_full_csr_comparison_kernel():
    import torch
    m = synth.ssymv_rmat(scale=14, batch=1 << 16, seed=31)
    rp, col = dev(m["rowptr"]), dev(m["col"])
    val, x = dev(m["val"].astype(np.float32)), dev(m["x"].astype(np.float32))
    frp, fcol, fval = systec.expand_csr(rp, col, val)
    _, counts = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), f32(m["x"]))
    assert fcol.numel() == counts["effective_nnz"]
    y = systec.spmv_csr(frp, fcol, fval, x).cpu().numpy()
    want, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), f32(m["x"]))
    assert rel_err(y, want) <= TOL32
    torch.cuda.synchronize()


# ------------------------------------------------------------------ MTTKRP --

def _mttkrp(t, B, bdtype="f32", algo="auto"):
    idx = [dev(a) for a in t["idx"]]
    val = dev(t["val"].astype(np.float32))
    if bdtype == "f32":
        Bd = dev(B.astype(np.float32))
    else:
        Bd = systec.quantize_bf16(dev(B.astype(np.float32)))
    return systec.mttkrp(idx, val, Bd, algo=algo).cpu().numpy()


def _oracle_mttkrp(t, B, bdtype="f32", row_mask=None):
    Bref = f32(B) if bdtype == "f32" else _bf16_round(B)
    return oracle.mttkrp(t["order"], t["dim"], t["idx"].T, f32(t["val"]), Bref,
                         row_mask=row_mask)


@pytest.mark.parametrize("order,dim,nnz", [(3, 300, 20011), (4, 120, 15013), (5, 60, 9001)])
@pytest.mark.parametrize("R", [1, 8, 16, 17, 32, 64, 100])
@pytest.mark.parametrize("bdtype", ["f32", "bf16"])
def test_mttkrp_matches_oracle(order, dim, nnz, R, bdtype):
    algo = "atomic"
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=1000 + order * 7 + R)
    B = synth.dense_uniform((dim, R), seed=R)
    print(f"mttkrp order={order} dim={dim} nnz={nnz} R={R} B={bdtype} algo={algo}", flush=True)
    C = _mttkrp(t, B, bdtype, algo)
    want, counts = _oracle_mttkrp(t, B, bdtype)
    assert all(h > 0 for h in counts["hist"])  # every equality pattern present
    assert rel_err(C, want) <= TOL32
    if bdtype == "bf16":
        full, _ = oracle.mttkrp(order, dim, t["idx"].T, t["val"], B)
        assert rel_err(C, full) <= TOL_BF16_E2E


@pytest.mark.parametrize("order", [3, 4, 5])
@pytest.mark.parametrize("algo", ["atomic", "auto"])
def test_mttkrp_all_diagonal_and_empty(order, algo):
    import torch
    dim, R = 700, 16
    diag = {"order": order, "dim": dim,
            "idx": np.stack([np.arange(dim, dtype=np.int32)] * order),
            "val": synth.dense_uniform(dim, seed=5)}
    B = synth.dense_uniform((dim, R), seed=6)
    C = _mttkrp(diag, B, algo=algo)
    want, _ = _oracle_mttkrp(diag, B)
    assert rel_err(C, want) <= TOL32
    empty = [torch.empty(0, dtype=torch.int32, device="cuda") for _ in range(order)]
    Ce = systec.mttkrp(empty, torch.empty(0, device="cuda"), dev(B.astype(np.float32)),
                       out=torch.full((dim, R), 3.0, device="cuda"), algo=algo)
    assert torch.count_nonzero(Ce).item() == 0


@pytest.mark.parametrize("order", [3, 5])
def test_mttkrp_long_leading_run(order):
    algo = "atomic"
    # every entry shares c1 = 0: one register-accumulated run across tiles
    dim = 40 if order == 3 else 14
    rest = np.array(list(itertools.combinations_with_replacement(range(dim), order - 1)),
                    dtype=np.int32)
    idx = np.concatenate([np.zeros((rest.shape[0], 1), np.int32), rest], axis=1)
    t = {"order": order, "dim": dim, "idx": np.ascontiguousarray(idx.T),
         "val": synth.dense_uniform(idx.shape[0], seed=8)}
    B = synth.dense_uniform((dim, 32), seed=9)
    assert idx.shape[0] > 512
    assert rel_err(_mttkrp(t, B, algo=algo), _oracle_mttkrp(t, B)[0]) <= TOL32


def test_mttkrp_order_invariance():
    algo = "auto"
    # the kernel does not rely on the list order for correctness
    t = synth.sym_coo(4, 200, 30000, 0.05, seed=77)
    B = synth.dense_uniform((200, 16), seed=78)
    C0 = _mttkrp(t, B, algo=algo)
    perm = np.random.Generator(np.random.PCG64(79)).permutation(30000)
    ts = dict(t, idx=np.ascontiguousarray(t["idx"][:, perm]), val=t["val"][perm])
    C1 = _mttkrp(ts, B, algo=algo)
    assert rel_err(C1, C0) <= TOL32


def test_mttkrp_oneshot_rejects_prepared_algorithms():
    t = synth.sym_coo(3, 50, 1000, 0.0, seed=5)
    B = dev(synth.dense_uniform((50, 8), seed=6).astype(np.float32))
    for algo in ("views", "lds"):
        with pytest.raises(systec.SystecError) as e:
            systec.mttkrp([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), B,
                          algo=algo)
        assert e.value.status_name == "SYSTEC_EINVAL"


# ---------------------------------------------------------- integer parts --

@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_expansion_stats_bit_exact(order):
    dim = {2: 4000, 3: 300, 4: 80, 5: 40}[order]
    t = synth.sym_coo(order, dim, 20000 if order > 2 else 30000, 0.02 if order == 2 else 0.3,
                      seed=300 + order)
    hist, eff = systec.expansion_stats([dev(a) for a in t["idx"]], t["dim"])
    r = oracle.expand(order, t["dim"], t["idx"].T)
    assert eff == r["effective_nnz"]
    assert hist == r["hist"]


def test_validation():
    good = synth.sym_coo(3, 100, 2000, 0.05, seed=5)
    systec.validate_coo([dev(a) for a in good["idx"]], 100)
    bad = good["idx"].copy()
    bad[:, [10, 11]] = bad[:, [11, 10]]  # list out of order
    with pytest.raises(systec.SystecError) as e:
        systec.validate_coo([dev(a) for a in bad], 100)
    assert e.value.status_name == "SYSTEC_ENONCANON"
    bad2 = good["idx"].copy()
    bad2[[0, 2], 5] = bad2[[2, 0], 5]  # tuple not ascending
    with pytest.raises(systec.SystecError):
        systec.validate_coo([dev(a) for a in bad2], 100)
    m = synth.ssymv_uniform(500, 5, seed=6)
    systec.validate_csr_upper(dev(m["rowptr"]), dev(m["col"]))
    col = m["col"].copy()
    col[m["rowptr"][10]] = 3  # below the diagonal in row 10
    with pytest.raises(systec.SystecError):
        systec.validate_csr_upper(dev(m["rowptr"]), dev(col))


def test_quantize_matches_oracle_rounding():
    import torch
    x = np.concatenate([synth.dense_uniform(100000, seed=3),
                        synth.dense_uniform(1000, seed=4) * 1e-38]).astype(np.float32)
    q = systec.quantize_bf16(dev(x)).to(torch.float64).cpu().numpy()
    np.testing.assert_array_equal(q, oracle.round_bf16(x))


# ------------------------------------------- non-symmetric comparison path --

@pytest.mark.parametrize("order,dim,nnz", [(3, 300, 20011), (4, 120, 15013), (5, 60, 9001)])
def test_expand_coo_bit_exact(order, dim, nnz):
    """The expansion behind the non-symmetric MTTKRP: the count, the grouping
    by the first index, and the multiset of expanded coordinates with their
    values, bit-exact against the oracle's enumeration."""
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=500 + order)
    idx = [dev(a) for a in t["idx"]]
    val32 = t["val"].astype(np.float32)
    fidx, fval = systec.expand_coo(idx, dev(val32), dim)
    r = oracle.expand(order, dim, t["idx"].T, coords_cap=10**7, per_entry=True)
    got = np.stack([a.cpu().numpy() for a in fidx], axis=1)
    assert got.shape[0] == r["effective_nnz"]
    assert np.all(np.diff(got[:, 0]) >= 0)  # grouped by the first index, rows ascending
    want = r["coords"]
    # coordinates: the same multiset (sorted lexicographically on both sides)
    go = np.lexsort(got.T[::-1])
    wo = np.lexsort(want.T[::-1])
    np.testing.assert_array_equal(got[go], want[wo])
    # values: each expanded coordinate carries the value of the stored entry
    # it expands (the oracle lists an entry's permutations consecutively)
    wval = np.repeat(val32, r["per_entry"])
    np.testing.assert_array_equal(fval.cpu().numpy()[go], wval[wo])


@pytest.mark.parametrize("order,dim,nnz", [(3, 300, 20011), (4, 120, 15013), (5, 60, 9001)])
@pytest.mark.parametrize("R", [1, 16, 17, 32, 100])
@pytest.mark.parametrize("bdtype", ["f32", "bf16"])
def test_nonsymmetric_mttkrp_matches_oracle(order, dim, nnz, R, bdtype):
    """MTTKRP over the expanded tensor (the paper's non-symmetric baseline)
    gives the oracle's result, element by element."""
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=600 + order * 7 + R)
    B = synth.dense_uniform((dim, R), seed=R + 1)
    print(f"non-symmetric mttkrp order={order} R={R} B={bdtype}", flush=True)
    idx = [dev(a) for a in t["idx"]]
    fidx, fval = systec.expand_coo(idx, dev(t["val"].astype(np.float32)), dim)
    Bd = dev(B.astype(np.float32))
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
    C = systec.mttkrp_full(fidx, fval, Bd).cpu().numpy()
    want, _ = _oracle_mttkrp(t, B, bdtype)
    Bref = f32(B) if bdtype == "f32" else _bf16_round(B)
    scale, _ = oracle.mttkrp(order, dim, t["idx"].T, np.abs(f32(t["val"])), np.abs(Bref))
    assert_elementwise(C, want, scale, TOL32, "non-symmetric mttkrp")
    assert rel_err(C, want) <= TOL32
    if bdtype == "bf16":
        full, _ = oracle.mttkrp(order, dim, t["idx"].T, t["val"], B)
        assert rel_err(C, full) <= TOL_BF16_E2E
