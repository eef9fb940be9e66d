"""Pins for the oracle's kernels beyond SSYMV, SYPRD and MTTKRP: the
Bellman-Ford (min, +) update, the 3-D TTM, MTTKRP of a partially symmetric
tensor and the symmetric CP step.

As in test_oracle_pins.py, nothing here compares the oracle with itself or
with the GPU library: the paper's printed TTM listings (tests/golden), dense
brute force with numpy, scipy's shortest paths and least squares, closed
forms, and enumeration properties. Integer-valued inputs keep FP64 exact.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_2406_09266_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _dense_sym_matrix(n, rowptr, col, val, absent=0.0):
    A = np.full((n, n), absent)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    A[rows, col] = val
    A[col, rows] = val
    return A


def _dense_sym_tensor(order, dim, idx, val, parts=None):
    """Dense tensor with v written at every arrangement of each stored tuple
    (every permutation, or with parts: permutations inside each part)."""
    parts = parts or [order]
    T = np.zeros((dim,) * order)
    starts = np.cumsum([0] + list(parts[:-1]))
    for e in range(idx.shape[0]):
        c = idx[e]
        pieces = [set(itertools.permutations(c[s:s + q])) for s, q in zip(starts, parts)]
        for combo in itertools.product(*pieces):
            T[sum(combo, ())] = val[e]
    return T


# ------------------------------------------------------------ Bellman-Ford --

def test_bellman_ford_equals_dense_min_plus():
    """y[i] = min_j (A[i,j] + d[j]) over the coordinates A stores (both
    triangles), +inf where none: bit-exact with integer values, negative
    weights included."""
    m = synth.ssymv_uniform(300, 6, seed=81)
    a = synth.integer_valued(m["col"].size, seed=82, low=-5, high=9)
    d = synth.integer_valued(300, seed=83, low=-20, high=20)
    d[::17] = np.inf  # unreachable vertices
    y, counts = oracle.bellman_ford(300, m["rowptr"], m["col"], a, d)
    A = _dense_sym_matrix(300, m["rowptr"], m["col"], a, absent=np.inf)
    np.testing.assert_array_equal(y, np.min(A + d[None, :], axis=1))
    rows = np.repeat(np.arange(300), np.diff(m["rowptr"]))
    assert counts["effective_nnz"] == 2 * m["col"].size - int(np.sum(rows == m["col"]))


def test_bellman_ford_empty_rows_stay_infinite():
    rowptr = np.array([0, 1, 1, 2, 2], np.int32)
    col = np.array([2, 2], np.int32)  # (0,2) and (2,2)
    y, _ = oracle.bellman_ford(4, rowptr, col, np.array([1.5, 4.0]), np.array([0.0, 1, 2, 3]))
    np.testing.assert_array_equal(y, [3.5, np.inf, 1.5, np.inf])


def test_bellman_ford_iterated_gives_shortest_paths():
    """Iterating the update from d = (0 at the source, +inf elsewhere), with a
    zero-weight self-loop on every vertex so a distance never grows, reaches
    the single-source shortest-path distances that scipy's Dijkstra finds."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    m = synth.ssymv_uniform(400, 3, seed=84, with_diagonal=False)
    n = m["n"]
    w = synth.dense_uniform(m["col"].size, seed=85, low=0.1, high=1.0)
    # add the zero diagonal: stored (i, i, 0) at the front of each row
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    r2 = np.concatenate([np.arange(n), rows])
    c2 = np.concatenate([np.arange(n), m["col"]])
    v2 = np.concatenate([np.zeros(n), w])
    o = np.lexsort((c2, r2))
    r2, c2, v2 = r2[o], c2[o].astype(np.int32), v2[o]
    rp2 = np.zeros(n + 1, np.int32)
    rp2[1:] = np.cumsum(np.bincount(r2, minlength=n))
    d = np.full(n, np.inf)
    d[0] = 0.0
    for _ in range(n):
        y, _ = oracle.bellman_ford(n, rp2, c2, v2, d)
        if np.array_equal(y, d):
            break
        d = y
    G = csr_matrix((w, (rows, m["col"])), shape=(n, n))
    ref = shortest_path(G, method="D", directed=False, indices=0)
    np.testing.assert_allclose(d, ref, rtol=1e-12)
    assert np.isinf(ref).sum() == np.isinf(d).sum()


# --------------------------------------------------------------------- TTM --

PATTERN3 = {"j<k<l": (1, 3, 6), "j=k<l": (2, 2, 5), "j<k=l": (0, 4, 4), "j=k=l": (3, 3, 3)}
SLOT = {"j": 0, "k": 1, "l": 2}


def test_ttm_matches_canonical_read_listing():
    """Sec. 3.1 TTM listing: for one stored entry of each pattern, C is the
    sum of the listing's assignments."""
    dim, R = 8, 4
    B = synth.integer_valued((dim, R), seed=91)
    table = read_table("ttm_listing_updates.txt")
    for pattern, tup in PATTERN3.items():
        v = -2.0
        want = np.zeros((dim, dim, R))
        for pat, o1, o2, br in table:
            if pat == pattern:
                want[tup[SLOT[o1]], tup[SLOT[o2]]] += v * B[tup[SLOT[br]]]
        C, counts = oracle.ttm3(dim, np.array([tup], np.int32), np.array([v]), B)
        np.testing.assert_array_equal(C, want, err_msg=pattern)
        assert counts["effective_nnz"] == sum(1 for r in table if r[0] == pattern)


def test_ttm_canonical_output_matches_output_symmetry_listing():
    """Sec. 3.2.1: with all indices distinct, the canonical triangle of the
    output (out1 <= out2) receives exactly the three updates of the listing
    after exploiting output symmetry, and the other triangle is its mirror."""
    dim, R = 8, 3
    B = synth.integer_valued((dim, R), seed=92)
    tup, v = PATTERN3["j<k<l"], 3.0
    want = np.zeros((dim, dim, R))
    for _, o1, o2, br in read_table("ttm_output_symmetry_updates.txt"):
        want[tup[SLOT[o1]], tup[SLOT[o2]]] += v * B[tup[SLOT[br]]]
    C, _ = oracle.ttm3(dim, np.array([tup], np.int32), np.array([v]), B)
    upper = np.triu(np.ones((dim, dim), bool))
    np.testing.assert_array_equal(C[upper], want[upper])
    np.testing.assert_array_equal(C, np.transpose(C, (1, 0, 2)))


@pytest.mark.parametrize("rep", [0.0, 0.3])
def test_ttm_equals_dense_brute_force(rep):
    dim, R = 9, 5
    t = synth.sym_coo(3, dim, 60, rep, seed=93)
    v = synth.integer_valued(t["val"].size, seed=94)
    B = synth.integer_valued((dim, R), seed=95)
    A = _dense_sym_tensor(3, dim, t["idx"].T, v)
    C, _ = oracle.ttm3(dim, t["idx"].T, v, B)
    np.testing.assert_array_equal(C, np.einsum("kjl,kr->jlr", A, B))


def test_ttm_rank_one_closed_form():
    """A = u (x) u (x) u gives C[j, l, r] = u_j u_l (u . B[:, r])."""
    dim, R = 7, 3
    u = synth.integer_valued(dim, seed=96)
    idx = np.array(list(itertools.combinations_with_replacement(range(dim), 3)), np.int32)
    v = u[idx[:, 0]] * u[idx[:, 1]] * u[idx[:, 2]]
    B = synth.integer_valued((dim, R), seed=97)
    C, _ = oracle.ttm3(dim, idx, v, B)
    np.testing.assert_array_equal(C, np.einsum("j,l,r->jlr", u, u, u @ B))


# ------------------------------------------------ partially symmetric MTTKRP --

PARTITIONS = [[2, 2], [3, 1], [1, 3], [2, 1, 1], [1, 2, 1], [2, 3], [3, 2], [1, 1, 1],
              [1, 1, 1, 1, 1], [4], [5]]


def _partial_canonical(parts, dim, count, seed):
    """Random tuples made canonical inside each part, unique, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = sum(parts)
    t = rng.integers(0, dim, (count, order))
    s = 0
    for q in parts:
        t[:, s:s + q] = np.sort(t[:, s:s + q], axis=1)
        s += q
    t = np.unique(t, axis=0).astype(np.int32)
    return t


def _einsum_partial(parts, T, F):
    order = T.ndim
    letters = "abcde"[:order]
    part_of = [q for q, size in enumerate(parts) for _ in range(size)]
    ops = [T] + [F[part_of[t]] for t in range(1, order)]
    spec = letters + "," + ",".join(f"{letters[t]}r" for t in range(1, order)) + "->ar"
    return np.einsum(spec, *ops)


@pytest.mark.parametrize("parts", PARTITIONS, ids=lambda p: "-".join(map(str, p)))
def test_partial_mttkrp_equals_dense_brute_force(parts):
    order = sum(parts)
    dim = {3: 7, 4: 6, 5: 5}[order]
    idx = _partial_canonical(parts, dim, 80, seed=100 + order)
    v = synth.integer_valued(idx.shape[0], seed=101)
    F = [synth.integer_valued((dim, 3), seed=102 + q) for q in range(len(parts))]
    T = _dense_sym_tensor(order, dim, idx, v, parts)
    C, counts = oracle.mttkrp_partial(parts, dim, idx, v, F)
    np.testing.assert_array_equal(C, _einsum_partial(parts, T, F))
    assert counts["effective_nnz"] == np.count_nonzero(T) or np.any(v == 0)


@pytest.mark.parametrize("order", [3, 4, 5])
def test_partial_mttkrp_one_part_is_full_symmetry(order):
    dim = {3: 12, 4: 10, 5: 9}[order]
    t = synth.sym_coo(order, dim, 150, 0.3, seed=110 + order)
    v = synth.integer_valued(t["val"].size, seed=111)
    B = synth.integer_valued((dim, 4), seed=112)
    C, k = oracle.mttkrp_partial([order], dim, t["idx"].T, v, [B])
    Cs, ks = oracle.mttkrp(order, dim, t["idx"].T, v, B)
    np.testing.assert_array_equal(C, Cs)
    assert k == ks


@pytest.mark.parametrize("parts", [[2, 2], [2, 1, 2], [1, 4], [3, 1]],
                         ids=lambda p: "-".join(map(str, p)))
def test_partial_expansion_covers_every_coordinate_once(parts):
    """Expanding every Pi-canonical tuple of [0, dim)^N yields dim^N
    coordinates; with v = 1 and unit factors each output row then counts
    dim^(N-1) coordinates, so none is missed or repeated."""
    order, dim = sum(parts), 4
    pieces = [list(itertools.combinations_with_replacement(range(dim), q)) for q in parts]
    idx = np.array([sum(c, ()) for c in itertools.product(*pieces)], np.int32)
    ones = [np.ones((dim, 1)) for _ in parts]
    C, counts = oracle.mttkrp_partial(parts, dim, idx, np.ones(idx.shape[0]), ones)
    assert counts["effective_nnz"] == dim ** order
    np.testing.assert_array_equal(C[:, 0], np.full(dim, float(dim ** (order - 1))))


def test_partial_noncanonical_sorted_inside_parts():
    parts, dim = [2, 2], 6
    idx = np.array([[4, 1, 0, 3], [1, 4, 3, 0]], np.int32)  # same orbit, both out of order
    F = [synth.integer_valued((dim, 2), seed=120 + q) for q in range(2)]
    C, k = oracle.mttkrp_partial(parts, dim, idx, np.array([1.0, 1.0]), F)
    C1, _ = oracle.mttkrp_partial(parts, dim, np.array([[1, 4, 0, 3]], np.int32),
                                  np.array([2.0]), F)
    np.testing.assert_array_equal(C, C1)
    assert k["noncanonical"] == 2


# ------------------------------------------------------------- CP step --

def _khatri_rao(B, copies):
    K = B
    for _ in range(copies - 1):
        K = np.einsum("ir,jr->ijr", K, B).reshape(-1, B.shape[1])
    return K


@pytest.mark.parametrize("order,R", [(3, 3), (4, 2), (3, 1)])
def test_cp_step_is_the_least_squares_update(order, R):
    """The one-factor update B_new = argmin_X || T_(1) - X KR^T ||_F, with KR
    the Khatri-Rao product of N-1 copies of B (the mode-1 unfolding of the
    CP model): solved by numpy's least squares on the dense tensor."""
    dim = 8 if order == 3 else 7
    t = synth.sym_coo(order, dim, 30, 0.2, seed=130 + order + R)
    B = synth.dense_uniform((dim, R), seed=131)
    r = oracle.cp_step(order, dim, t["idx"].T, t["val"], B)
    T = _dense_sym_tensor(order, dim, t["idx"].T, t["val"])
    T1 = T.reshape(dim, -1)
    KR = _khatri_rao(B, order - 1)
    X = np.linalg.lstsq(KR, T1.T, rcond=None)[0].T
    np.testing.assert_allclose(r["B_new"], X, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("order", [3, 4, 5])
def test_cp_fit_terms_equal_dense(order):
    dim, R = {3: 8, 4: 7, 5: 7}[order], 3
    t = synth.sym_coo(order, dim, 20, 0.3, seed=140 + order)
    B = synth.dense_uniform((dim, R), seed=141)
    r = oracle.cp_step(order, dim, t["idx"].T, t["val"], B)
    T = _dense_sym_tensor(order, dim, t["idx"].T, t["val"])
    M = np.zeros_like(T)
    for q in range(R):
        b = B[:, q]
        outer = b
        for _ in range(order - 1):
            outer = np.multiply.outer(outer, b)
        M += outer
    np.testing.assert_allclose(r["norm_T2"], np.sum(T * T), rtol=1e-12)
    np.testing.assert_allclose(r["inner"], np.sum(T * M), rtol=1e-12)
    np.testing.assert_allclose(r["norm_M2"], np.sum(M * M), rtol=1e-12)
    np.testing.assert_allclose(r["resid2"], np.sum((T - M) ** 2), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("order", [3, 4, 5])
def test_cp_rank_one_fixed_point(order):
    """T = u^(x N) with B = u: MTTKRP gives u (u.u)^(N-1) exactly (integers),
    the update returns u and the residual is zero, to the rounding of the
    solve."""
    dim = 6
    u = synth.integer_valued(dim, seed=150, low=1, high=3)
    idx = np.array(list(itertools.combinations_with_replacement(range(dim), order)), np.int32)
    v = np.prod(u[idx], axis=1)
    r = oracle.cp_step(order, dim, idx, v, u.reshape(-1, 1))
    np.testing.assert_array_equal(r["C"][:, 0], u * (u @ u) ** (order - 1))
    np.testing.assert_allclose(r["B_new"][:, 0], u, rtol=1e-14)
    assert r["norm_T2"] == (u @ u) ** order == r["inner"] == r["norm_M2"]
    assert r["resid2"] == 0.0


def test_cp_rank_one_update_is_the_power_step():
    """R = 1: b_new = T b^(N-1) / (b . b)^(N-1), the symmetric power step."""
    dim, order = 8, 4
    t = synth.sym_coo(order, dim, 50, 0.3, seed=160)
    b = synth.dense_uniform(dim, seed=161)
    r = oracle.cp_step(order, dim, t["idx"].T, t["val"], b.reshape(-1, 1))
    T = _dense_sym_tensor(order, dim, t["idx"].T, t["val"])
    Tb = np.einsum("iklm,k,l,m->i", T, b, b, b)
    np.testing.assert_allclose(r["B_new"][:, 0], Tb / (b @ b) ** 3, rtol=1e-12)
