"""GPU parity of the Bellman-Ford update y[i] = min_j (A[i,j] + d[j]) over a
symmetric matrix stored by its upper triangle (the (min, +) form of SSYMV),
one-shot and prepared, against the FP64 oracle.

The minimum is exact on both sides: FP32 rounding is monotonic, so the
minimum of the GPU's FP32 sums a + d is the FP32 rounding of the oracle's
FP64 minimum whenever the FP64 sums are exact (always here: the inputs are
FP32 values of similar magnitude). The test therefore asks for bit-exact
equality with the oracle's result rounded to FP32, +inf included."""
import numpy as np
import pytest

import oracle
import paper_2406_09266_amd as systec
from paper_2406_09266_amd import synth

from gpu_util import dev, f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _distances(n, seed, unreachable=0.1, negative=False):
    """Path lengths: U(0, 4) (or N(0,1) when negative values are allowed),
    with a fraction set to +inf (not reached yet)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal(n) if negative else rng.uniform(0.0, 4.0, n)
    d[rng.random(n) < unreachable] = np.inf
    return d.astype(np.float32)


CASES = {
    "small_n2000": lambda: synth.workload("ssymv_small"),
    "uniform_n5003_ragged": lambda: synth.ssymv_uniform(5003, 9, seed=11),
    "rmat_scale14_hubs": lambda: synth.ssymv_rmat(scale=14, batch=1 << 16, seed=12),
    "rmat_scale16_relabel": lambda: synth.ssymv_rmat(scale=16, batch=1 << 18, seed=13,
                                                     relabel=True),
    "diagonal_only": lambda: synth.ssymv_uniform(3000, 0, seed=14),
    "random_degree_n40000": lambda: synth.ssymv_random_degree(40000, 12, seed=15),
}


def _want(m, val32, d):
    y, counts = oracle.bellman_ford(m["n"], m["rowptr"], m["col"], val32.astype(np.float64),
                                    d.astype(np.float64))
    return y.astype(np.float32), counts


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("negative", [False, True])
@pytest.mark.parametrize("form", ["oneshot", "prepared", "prepared_relabeled"])
def test_bellman_ford_matches_oracle(case, negative, form):
    m = CASES[case]()
    n = m["n"]
    print(f"bellman-ford case={case} negative={negative} form={form} n={n}", flush=True)
    val32 = m["val"].astype(np.float32)
    if negative:  # edge lengths of either sign
        val32 = (val32 - 0.5).astype(np.float32)
    d = _distances(n, seed=n + 7, negative=negative)
    want, counts = _want(m, val32, d)
    rp, col, val = dev(m["rowptr"]), dev(m["col"]), dev(val32)
    dd = dev(d)
    if form == "oneshot":
        y = systec.bellman_ford(rp, col, val, dd)
    else:
        A = systec.Tensor.from_csr(rp, col, val, relabel=(form == "prepared_relabeled"))
        y = A.bellman_ford(dd)
        assert A.effective_nnz == counts["effective_nnz"]
    got = y.cpu().numpy()
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("form", ["oneshot", "prepared"])
def test_bellman_ford_empty_and_isolated(form):
    """No stored coordinate: every y[i] is +inf. One stored diagonal of
    length 0: it carries d over."""
    import torch
    n = 37
    rp = dev(np.zeros(n + 1, dtype=np.int32))
    empty_i = torch.empty(0, dtype=torch.int32, device="cuda")
    empty_f = torch.empty(0, dtype=torch.float32, device="cuda")
    d = dev(np.arange(n, dtype=np.float32))
    out = torch.full((n,), 5.0, device="cuda")
    if form == "oneshot":
        y = systec.bellman_ford(rp, empty_i, empty_f, d, out=out)
    else:
        y = systec.Tensor.from_csr(rp, empty_i, empty_f).bellman_ford(d, out=out)
    assert bool(torch.isinf(y).all()) and bool((y > 0).all())
    # a zero diagonal everywhere plus one edge (0, 5) of length 1: y = min(d, ...)
    rowptr = np.concatenate([[0], np.arange(2, n + 2)]).astype(np.int32)
    cols = np.concatenate([[0, 5], np.arange(1, n)]).astype(np.int32)
    vals = np.zeros(n + 1, np.float32)
    vals[1] = 1.0
    m = {"n": n, "rowptr": rowptr, "col": cols}
    dn = np.arange(n, dtype=np.float32)[::-1].copy()
    want, _ = _want(m, vals, dn)
    if form == "oneshot":
        got = systec.bellman_ford(dev(rowptr), dev(cols), dev(vals), dev(dn)).cpu().numpy()
    else:
        A = systec.Tensor.from_csr(dev(rowptr), dev(cols), dev(vals))
        got = A.bellman_ford(dev(dn)).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    assert got[0] == min(dn[0], 1.0 + dn[5])


def test_bellman_ford_iterates_to_shortest_paths():
    """Repeated updates from a single source converge to the shortest path
    lengths that scipy computes (a zero diagonal carries the lengths over)."""
    import scipy.sparse
    import scipy.sparse.csgraph
    m = synth.ssymv_uniform(3000, 4, seed=21)
    n = m["n"]
    val32 = (m["val"].astype(np.float32) ** 2 + 0.01).astype(np.float32)
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    diag = rows == m["col"]
    val32[diag] = 0.0
    A = systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]), dev(val32), relabel=True)
    d = np.full(n, np.inf, np.float32)
    d[0] = 0.0
    dd = dev(d)
    for _ in range(200):
        nd = A.bellman_ford(dd)
        if bool((nd == dd).all()):
            break
        dd = nd
    up = scipy.sparse.csr_matrix((val32[~diag].astype(np.float64),
                                  (rows[~diag], m["col"][~diag])), shape=(n, n))
    ref = scipy.sparse.csgraph.dijkstra(up, directed=False, indices=0)
    got = dd.cpu().numpy().astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.max(np.abs(got[fin] - ref[fin]) / np.maximum(ref[fin], 1e-30)) <= 1e-5
