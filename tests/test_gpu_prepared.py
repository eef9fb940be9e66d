"""GPU parity of the prepared operands (panel format for matrices, slot views
for tensors) against the FP64 oracle; same tolerances as test_gpu_parity."""
import numpy as np
import pytest

import oracle
import paper_2406_09266_amd as systec
from paper_2406_09266_amd import synth

from gpu_util import assert_elementwise, dev, f32, rel_err, wide_step_matrix

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _x(m, xdtype):
    x = dev(m["x"].astype(np.float32))
    if xdtype == "bf16":
        return systec.quantize_bf16(x), oracle.round_bf16(m["x"].astype(np.float32))
    return x, f32(m["x"])


MATRICES = {
    "small_n2000": lambda: synth.workload("ssymv_small"),
    "uniform_n40000_ragged_panels": lambda: synth.ssymv_uniform(40001, 9, seed=51),
    "rmat_scale16": lambda: synth.ssymv_rmat(scale=16, batch=1 << 18, seed=52),
    "rmat_scale15_relabel": lambda: synth.ssymv_rmat(scale=15, batch=1 << 17, seed=53,
                                                     relabel=True),
    "diagonal_only": lambda: synth.ssymv_uniform(20000, 0, seed=54),
}


@pytest.mark.parametrize("case", sorted(MATRICES))
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_ssymv(case, xdtype):
    m = MATRICES[case]()
    print(f"prepared ssymv case={case} x={xdtype} n={m['n']} nnz={m['col'].size}", flush=True)
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)))
    x, xref = _x(m, xdtype)
    y = A.ssymv(x).cpu().numpy()
    want, counts = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(y, want) <= TOL32
    assert A.effective_nnz == counts["effective_nnz"] and A.nnz == m["col"].size
    assert A.order == 2 and A.bytes > 0
    # a second call on the same handle gives the same result within tolerance
    y2 = A.ssymv(x).cpu().numpy()
    assert rel_err(y2, y) <= TOL32
    A.close()


@pytest.mark.parametrize("case", ["small_n2000", "uniform_n40000_ragged_panels", "rmat_scale16",
                                  "diagonal_only"])
@pytest.mark.parametrize("relabel", [True, False])
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_ssymv_vertex_order(case, relabel, xdtype):
    """The matrix stored with its vertices ordered by degree (x permuted in,
    y permuted out) or in the caller's order gives the oracle's result."""
    m = MATRICES[case]()
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=relabel)
    x, xref = _x(m, xdtype)
    y = A.ssymv(x).cpu().numpy()
    want, counts = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(y, want) <= TOL32
    assert A.effective_nnz == counts["effective_nnz"]
    A.close()


@pytest.mark.parametrize("relabel", [True, False])
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_syprd(relabel, xdtype):
    """x^T A x over the prepared format (vertex or degree order) against the
    oracle, on a matrix of several panels and on one with a ragged tail."""
    for m in (synth.ssymv_rmat(scale=15, batch=1 << 17, seed=57),
              synth.ssymv_uniform(40001, 9, seed=58)):
        A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]),
                                   dev(m["val"].astype(np.float32)), relabel=relabel)
        x, xref = _x(m, xdtype)
        s = A.syprd(x).item()
        want, scale, _ = oracle.syprd(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
        assert abs(s - want) <= TOL32 * scale
        A.close()


@pytest.mark.parametrize("relabel", [True, False])
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_stored_order_calls(relabel, xdtype):
    """x and y in the stored vertex order: the same kernel on the same
    permuted x, so y_stored equals the caller-order result permuted (up to
    the order of the FP32 atomic additions), and the scalar, which has no
    atomics, equals it exactly."""
    import torch
    m = synth.ssymv_rmat(scale=14, batch=1 << 16, seed=59)
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=relabel)
    x, _ = _x(m, xdtype)
    perm = A.vertex_order()
    pl = (perm if perm is not None else torch.arange(m["n"], device="cuda")).long()
    xs = x[pl].contiguous()
    y = A.ssymv(x)
    ys = A.ssymv(xs, stored_order=True)
    assert rel_err(ys.cpu().numpy(), y[pl].cpu().numpy()) <= TOL32
    assert A.syprd(xs, stored_order=True).item() == A.syprd(x).item()
    A.close()


@pytest.mark.parametrize("relabel", [True, False])
def test_prepared_ssymv_reports_vertex_order(relabel):
    """The stored order is a permutation by descending degree, ties in vertex
    order (degree counted on the CPU from the stored triangle)."""
    m = synth.ssymv_rmat(scale=12, batch=1 << 15, seed=56)
    n = m["n"]
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=relabel)
    perm = A.vertex_order()
    A.close()
    if not relabel:
        assert perm is None
        return
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    col = m["col"].astype(np.int64)
    deg = np.bincount(rows, minlength=n) + np.bincount(col[col != rows], minlength=n)
    assert np.array_equal(perm, np.argsort(-deg, kind="stable"))




@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_ssymv_unaligned_x(xdtype):
    """x one element past a 16-byte boundary: the panels' x slices are staged
    element by element instead of in 16-byte pieces."""
    import torch
    m = synth.ssymv_uniform(40001, 9, seed=59)
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=False)  # x reaches the panel kernels as given
    x, xref = _x(m, xdtype)
    buf = torch.empty(m["n"] + 1, dtype=x.dtype, device="cuda")
    buf[1:] = x
    xu = buf[1:]
    assert xu.data_ptr() % 16 != 0
    y = A.ssymv(xu).cpu().numpy()
    want, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(y, want) <= TOL32
    s = A.syprd(xu).item()
    swant, scale, _ = oracle.syprd(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert abs(s - swant) <= TOL32 * scale
    A.close()


def test_prepared_ssymv_empty_rows_and_panels():
    import torch
    # rows only in the last panel; earlier panels empty
    n = 140000
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[n - 100:] = np.arange(0, 101, dtype=np.int32)  # rows n-100.. hold one entry each
    cols = np.arange(n - 100, n, dtype=np.int32)           # on the diagonal
    m = {"n": n, "rowptr": rowptr, "col": cols, "val": synth.dense_uniform(100, seed=1),
         "x": synth.dense_uniform(n, seed=2)}
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)))
    x, xref = _x(m, "f32")
    y = A.ssymv(x).cpu().numpy()
    want, _ = oracle.ssymv(n, m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(y, want) <= TOL32
    # nnz = 0
    E = systec.Tensor.from_csr(dev(np.zeros(11, np.int32)), torch.empty(0, dtype=torch.int32,
                               device="cuda"), torch.empty(0, device="cuda"))
    ye = E.ssymv(dev(np.ones(10, np.float32)), out=torch.full((10,), 5.0, device="cuda"))
    assert torch.count_nonzero(ye).item() == 0


def _wide_steps(m, H=8192):
    """Steps of 64 entries in the vertex-order panel layout (panels of H rows,
    entries sorted by column, padded to 512 with the last column) whose
    columns span 2^(32 - log2 H) or more."""
    rows = np.repeat(np.arange(m["n"]), np.diff(m["rowptr"]))
    p = rows // H
    wide = 0
    for q in np.unique(p):
        c = np.sort(m["col"][p == q])
        c = np.r_[c, np.full((-c.size) % 512, c[-1])].reshape(-1, 64)
        wide += int(np.count_nonzero(c[:, -1] - c[:, 0] >= 1 << (32 - 13)))
    return wide


@pytest.mark.parametrize("relabel", [True, False])
@pytest.mark.parametrize("xdtype", ["f32", "bf16"])
def test_prepared_wide_steps(relabel, xdtype):
    """SSYMV and SYPRD where some steps' columns overflow the packed offsets."""
    m = wide_step_matrix()
    assert _wide_steps(m) > 100  # the fallback path is exercised (vertex order)
    print(f"prepared wide steps relabel={relabel} x={xdtype} n={m['n']} nnz={m['col'].size}",
          flush=True)
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=relabel)
    x, xref = _x(m, xdtype)
    y = A.ssymv(x).cpu().numpy()
    want, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(y, want) <= TOL32
    absref, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], np.abs(f32(m["val"])), np.abs(xref))
    assert_elementwise(y, want, absref, TOL32)
    s = A.syprd(x).item()
    swant, scale, _ = oracle.syprd(m["n"], m["rowptr"], m["col"], f32(m["val"]), xref)
    assert abs(s - swant) <= TOL32 * scale
    A.close()


@pytest.mark.parametrize("relabel", [True, False])
def test_prepared_edge_cases_syprd_and_vertex_order(relabel):
    """Entries only in the last of nine panels (all in the first panel once
    relabeled), and a matrix with no entries: SSYMV and SYPRD against the
    oracle, SYPRD of the empty matrix exactly zero."""
    import torch
    n = 140000
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[n - 100:] = np.arange(0, 101, dtype=np.int32)
    cols = np.arange(n - 100, n, dtype=np.int32)
    cols[:50] = n - 1  # half of them off the diagonal, all in the last column
    m = {"n": n, "rowptr": rowptr, "col": cols, "val": synth.dense_uniform(100, seed=5),
         "x": synth.dense_uniform(n, seed=6)}
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
                               relabel=relabel)
    assert (A.vertex_order() is not None) == relabel
    x, xref = _x(m, "f32")
    want, _ = oracle.ssymv(n, m["rowptr"], m["col"], f32(m["val"]), xref)
    assert rel_err(A.ssymv(x).cpu().numpy(), want) <= TOL32
    s = A.syprd(x).item()
    want_s, scale, _ = oracle.syprd(n, m["rowptr"], m["col"], f32(m["val"]), xref)
    assert abs(s - want_s) <= TOL32 * scale
    A.close()
    E = systec.Tensor.from_csr(dev(np.zeros(11, np.int32)), torch.empty(0, dtype=torch.int32,
                               device="cuda"), torch.empty(0, device="cuda"), relabel=relabel)
    assert E.vertex_order() is None  # nothing to relabel
    assert E.syprd(dev(np.ones(10, np.float32))).item() == 0.0
    E.close()


def test_prepared_rejects_noncanonical():
    m = synth.ssymv_uniform(300, 5, seed=3)
    col = m["col"].copy()
    col[m["rowptr"][7]] = 2
    with pytest.raises(systec.SystecError) as e:
        systec.Tensor.from_csr(dev(m["rowptr"]), dev(col), dev(m["val"].astype(np.float32)))
    assert e.value.status_name == "SYSTEC_ENONCANON"
    t = synth.sym_coo(3, 50, 500, 0.1, seed=4)
    bad = t["idx"].copy()
    bad[:, [3, 4]] = bad[:, [4, 3]]
    with pytest.raises(systec.SystecError):
        systec.Tensor.from_coo([dev(a) for a in bad], dev(t["val"].astype(np.float32)), 50)


@pytest.mark.parametrize("order,dim,nnz", [(3, 400, 30011), (4, 150, 20021), (5, 70, 12007)])
@pytest.mark.parametrize("R", [1, 16, 32, 70])
@pytest.mark.parametrize("bdtype", ["f32", "bf16"])
@pytest.mark.parametrize("algo", ["views", "lds", "atomic"])
def test_prepared_mttkrp(order, dim, nnz, R, bdtype, algo):
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=2000 + order * 11 + R)
    B = synth.dense_uniform((dim, R), seed=R + 1)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    Bd = dev(B.astype(np.float32))
    Bref = f32(B)
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
        Bref = oracle.round_bf16(B.astype(np.float32))
    C = T.mttkrp(Bd, algo=algo).cpu().numpy()
    want, counts = oracle.mttkrp(order, dim, t["idx"].T, f32(t["val"]), Bref)
    assert rel_err(C, want) <= TOL32
    assert T.effective_nnz == counts["effective_nnz"]
    T.close()


@pytest.mark.parametrize("order,dim,nnz", [(3, 400, 30011), (4, 150, 20021), (5, 70, 12007)])
@pytest.mark.parametrize("R,bdtype", [(6, "bf16"), (8, "bf16"), (16, "bf16"), (24, "bf16"),
                                      (64, "bf16"), (72, "bf16"), (136, "bf16"), (2, "f32"),
                                      (4, "f32"), (12, "f32"), (32, "f32"), (64, "f32")])
def test_prepared_mttkrp_vector_lanes(order, dim, nnz, R, bdtype):
    """Slot views with vector lanes (2, 4 or 8 columns per lane, R even, runs
    of 75 to 171 entries per index): one to sixteen lanes per row, idle lanes
    when R/V is not a power of two, and 64-column blocks with a ragged last
    block of another lane width."""
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=3000 + order * 13 + R)
    B = synth.dense_uniform((dim, R), seed=R + 7)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    Bd = dev(B.astype(np.float32))
    Bref = f32(B)
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
        Bref = oracle.round_bf16(B.astype(np.float32))
    C = T.mttkrp(Bd, algo="views").cpu().numpy()
    want, _ = oracle.mttkrp(order, dim, t["idx"].T, f32(t["val"]), Bref)
    assert rel_err(C, want) <= TOL32
    T.close()


@pytest.mark.parametrize("order,dim,nnz", [(3, 20000, 30011), (4, 5000, 20021)])
@pytest.mark.parametrize("R,bdtype", [(8, "bf16"), (32, "bf16"), (16, "f32"), (40, "f32")])
def test_prepared_mttkrp_short_runs(order, dim, nnz, R, bdtype):
    """Fewer than 64 stored entries per index (runs of one to four entries
    per output row): vector lanes summing the short rows of an iteration
    across lane groups up to 16 columns, one lane per column above."""
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.05, seed=4000 + order + R)
    B = synth.dense_uniform((dim, R), seed=R + 11)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    Bd = dev(B.astype(np.float32))
    Bref = f32(B)
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
        Bref = oracle.round_bf16(B.astype(np.float32))
    C = T.mttkrp(Bd, algo="views").cpu().numpy()
    want, _ = oracle.mttkrp(order, dim, t["idx"].T, f32(t["val"]), Bref)
    assert rel_err(C, want) <= TOL32
    # where all of B fits LDS the automatic choice would take the lane form,
    # which short runs exclude: it falls back to the views
    assert rel_err(T.mttkrp(Bd).cpu().numpy(), want) <= TOL32
    T.close()


@pytest.mark.parametrize("order", [3, 5])
def test_prepared_mttkrp_all_diagonal(order):
    dim = 900
    idx = np.stack([np.arange(dim, dtype=np.int32)] * order)
    val = synth.dense_uniform(dim, seed=9)
    B = synth.dense_uniform((dim, 16), seed=10)
    T = systec.Tensor.from_coo([dev(a) for a in idx], dev(val.astype(np.float32)), dim)
    C = T.mttkrp(dev(B.astype(np.float32))).cpu().numpy()
    want, _ = oracle.mttkrp(order, dim, idx.T, f32(val), f32(B))
    assert rel_err(C, want) <= TOL32


@pytest.mark.parametrize("order,dim,R,bdtype", [
    (5, 5000, 16, "bf16"),    # the 5-D workload's shape: one 16-column slice
    (3, 10000, 8, "bf16"),    # near the LDS limit: one 8-column slice
    (4, 9000, 3, "f32"),      # FP32 B, ragged slice (4 columns, 3 used)
    (3, 2000, 100, "bf16"),   # two 64-column slices, ragged last slice
    (4, 600, 40, "f32"),      # FP32 B, one 64-column slice (40 used)
    (5, 30, 16, "f32"),       # fewer entries than workgroups x lane groups
    (4, 1200, 32, "f32"),     # all of B in LDS (153,600 B), FP32, 32 columns
    (3, 3000, 16, "f32"),     # all of B in LDS, views ending inside a wave tile
])
def test_prepared_mttkrp_lds_shapes(order, dim, R, bdtype):
    nnz = {5000: 200003, 10000: 150001, 9000: 120007, 2000: 50021, 600: 40009, 30: 3001,
           1200: 90017, 3000: 200019}[dim]
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.05, seed=2000 + dim)
    B = synth.dense_uniform((dim, R), seed=dim)
    print(f"prepared mttkrp lds order={order} dim={dim} nnz={nnz} R={R} B={bdtype}", flush=True)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    Bd = dev(B.astype(np.float32))
    Bref = f32(B)
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
        Bref = oracle.round_bf16(B.astype(np.float32))
    want, _ = oracle.mttkrp(order, dim, t["idx"].T, f32(t["val"]), Bref)
    scale, _ = oracle.mttkrp(order, dim, t["idx"].T, np.abs(f32(t["val"])), np.abs(Bref))
    for algo in ("lds", "views", "auto"):
        C = T.mttkrp(Bd, algo=algo).cpu().numpy()
        assert_elementwise(C, want, scale, TOL32, f"lds shape {algo}")
        assert rel_err(C, want) <= TOL32
    T.close()


@pytest.mark.parametrize("special", ["none", "tiny", "huge"])
@pytest.mark.parametrize("order", [3, 5])
def test_prepared_mttkrp_lane_form_half_staging(order, special):
    """The one-lane-per-entry form with a BF16 factor: staged as FP16 when
    every value converts exactly, as BF16 when one does not (a value below
    2^-17 or above 65,504); both against the oracle, element by element."""
    dim, R = 900, 16
    t = synth.sym_coo(order, dim, 120011, repeat_frac=0.1, seed=77 + order)
    B = synth.dense_uniform((dim, R), seed=78)
    B[B == 0] = 0.5
    B = np.where(np.abs(B) < 1e-3, 1e-3, B)  # all in FP16's exact range ...
    if special == "tiny":
        B[17, 3] = 3.0e-7  # ... except one value
    elif special == "huge":
        B[dim - 1, R - 1] = -1.5e5
    Bref = oracle.round_bf16(B.astype(np.float32))
    with np.errstate(over="ignore"):
        exact = np.all(Bref.astype(np.float16).astype(np.float32) == Bref)
    assert exact == (special == "none")
    print(f"lane form order={order} special={special}", flush=True)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    Bd = systec.quantize_bf16(dev(B.astype(np.float32)))
    want, _ = oracle.mttkrp(order, dim, t["idx"].T, f32(t["val"]), Bref)
    scale, _ = oracle.mttkrp(order, dim, t["idx"].T, np.abs(f32(t["val"])), np.abs(Bref))
    for algo in ("lds", "auto"):
        C = T.mttkrp(Bd, algo=algo).cpu().numpy()
        assert_elementwise(C, want, scale, TOL32, f"lane form {special} {algo}")
    T.close()


def test_prepared_mttkrp_lds_rejects_large_index_space():
    import torch
    t = synth.sym_coo(3, 100000, 1000, 0.0, seed=5)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)),
                               100000)
    Bh = synth.dense_uniform((100000, 16), seed=6)
    B = dev(Bh.astype(np.float32))
    with pytest.raises(systec.SystecError) as e:
        T.mttkrp(B, algo="lds")
    assert e.value.status_name == "SYSTEC_EINVAL"
    assert systec.mttkrp_choose(100000, 16, False, True) == "views"
    assert systec.mttkrp_choose(5000, 16, True, True) == "lds"  # all of B fits LDS
    assert systec.mttkrp_choose(5000, 16, False, True) == "views"  # 320,000 B does not
    assert systec.mttkrp_choose(5000, 12, True, True) == "views"  # R outside 8, 16, 32
    assert systec.mttkrp_choose(5000, 16, True, False) == "atomic"
    C = T.mttkrp(B)  # the automatic choice falls back to the views
    torch.cuda.synchronize()
    want, _ = oracle.mttkrp(3, 100000, t["idx"].T, f32(t["val"]), f32(Bh))
    assert rel_err(C.cpu().numpy(), want) <= TOL32
    T.close()
