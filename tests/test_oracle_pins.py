"""Pins for the FP64 oracle: what the paper and the mathematics fix.

None of these compares the oracle with itself or with the GPU library. Each
checks it against something independent: the paper's printed worked examples
(tests/golden), dense brute force built with itertools and numpy.einsum,
closed forms, scipy, and enumeration / invariance properties. Integer-valued
inputs make every FP64 result exact, so most checks are bit-exact.
"""
import itertools
import os
from fractions import Fraction

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
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


# concrete tuples for each equality pattern of a sorted 3-tuple (i, k, l)
PATTERN3 = {"i<k<l": (1, 3, 6), "i=k<l": (2, 2, 5), "i<k=l": (0, 4, 4), "i=k=l": (3, 3, 3)}
SLOT3 = {"i": 0, "k": 1, "l": 2}


def _single(order, tup, v, dim):
    idx = np.array(tup, dtype=np.int32).reshape(1, order)
    return idx, np.array([v], dtype=np.float64)


# ---------------------------------------------------------------- golden ----

def test_mttkrp3_matches_normalized_listing():
    """Sec. 4.3 normalized MTTKRP listing: per pattern, the updates it makes."""
    dim, R = 7, 5
    B = synth.integer_valued((dim, R), seed=11)
    table = read_table("mttkrp3_normalized_updates.txt")
    for pattern, tup in PATTERN3.items():
        v = 3.0
        expected = np.zeros((dim, R))
        for pat, out, count in table:
            if pat != pattern:
                continue
            s = SLOT3[out]
            others = [t for t in range(3) if t != s]
            expected[tup[s]] += int(count) * v * B[tup[others[0]]] * B[tup[others[1]]]
        idx, val = _single(3, tup, v, dim)
        C, _ = oracle.mttkrp(3, dim, idx, val, B)
        np.testing.assert_array_equal(C, expected, err_msg=pattern)


def test_mttkrp3_matches_split_nest_listing():
    """Sec. 4.3 split loop nests (distributive grouping + diagonal split)."""
    dim, R = 8, 4
    B = synth.integer_valued((dim, R), seed=12)
    table = read_table("mttkrp3_split_nests.txt")
    for pattern, tup in PATTERN3.items():
        v = -2.0
        expected = np.zeros((dim, R))
        for pat, out, coef in table:
            if pat != pattern:
                continue
            s = SLOT3[out]
            o = [t for t in range(3) if t != s]
            expected[tup[s]] += int(coef) * v * B[tup[o[0]]] * B[tup[o[1]]]
        idx, val = _single(3, tup, v, dim)
        C, _ = oracle.mttkrp(3, dim, idx, val, B)
        np.testing.assert_array_equal(C, expected, err_msg=pattern)


def test_mttkrp3_matches_lookup_table_factors():
    """Sec. 4.2.5: uniform factor per pattern applied to one update per slot."""
    dim, R = 7, 3
    B = synth.integer_valued((dim, R), seed=13)
    factors = {p: float(Fraction(f)) for p, f in read_table("lut_factors_3d.txt")}
    for pattern, tup in PATTERN3.items():
        v = 6.0  # a multiple of 3 keeps 1/3 exact
        expected = np.zeros((dim, R))
        for s in range(3):
            o = [t for t in range(3) if t != s]
            expected[tup[s]] += factors[pattern] * v * B[tup[o[0]]] * B[tup[o[1]]]
        idx, val = _single(3, tup, v, dim)
        C, _ = oracle.mttkrp(3, dim, idx, val, B)
        np.testing.assert_allclose(C, expected, rtol=0, atol=1e-12, err_msg=pattern)


def test_ssymv_matches_figure():
    """Sec. 3.1 figure: i<j gives two updates, i==j one."""
    n = 5
    x = np.array([2.0, -1.0, 3.0, 5.0, -4.0])
    a = 1.5
    names = {"i": 1, "j": 3}
    for pattern, rows in itertools.groupby(read_table("ssymv_updates.txt"), key=lambda r: r[0]):
        i, j = (1, 3) if pattern == "i<j" else (2, 2)
        names = {"i": i, "j": j}
        expected = np.zeros(n)
        for _, out, inp, count in rows:
            expected[names[out]] += int(count) * a * x[names[inp]]
        rowptr = np.zeros(n + 1, dtype=np.int32)
        rowptr[i + 1:] = 1
        y, counts = oracle.ssymv(n, rowptr, [j], [a], x)
        np.testing.assert_array_equal(y, expected, err_msg=pattern)


def test_syprd_matches_listing():
    """Sec. 3.2.2 SYPRD listings: 2 x_i a x_j off the diagonal, once on it."""
    n = 4
    x = np.array([2.0, -1.0, 3.0, 5.0])
    a = -0.5
    for pattern, coef in read_table("syprd_updates.txt"):
        i, j = (0, 2) if pattern == "i<j" else (3, 3)
        rowptr = np.zeros(n + 1, dtype=np.int32)
        rowptr[i + 1:] = 1
        s, sa, _ = oracle.syprd(n, rowptr, [j], [a], x)
        assert s == int(coef) * x[i] * a * x[j]
        assert sa == abs(s)


def test_update_counts_match_ttm_listing():
    """Sec. 3.1: 6 / 3 / 3 / 1 updates per canonical read of a 3-index tensor."""
    pat_tuple = {"j<k<l": (1, 3, 6), "j=k<l": (2, 2, 5), "j<k=l": (0, 4, 4), "j=k=l": (3, 3, 3)}
    for pattern, updates in read_table("ttm_update_counts.txt"):
        r = oracle.expand(3, 8, np.array([pat_tuple[pattern]]), per_entry=True)
        assert int(r["per_entry"][0]) == int(updates), pattern


# ----------------------------------------------------------- enumeration ----

def _all_multisets(dim, order):
    return np.array(list(itertools.combinations_with_replacement(range(dim), order)),
                    dtype=np.int32)


@pytest.mark.parametrize("order,dim", [(2, 9), (3, 8), (4, 7), (5, 8)])
def test_expansion_covers_every_coordinate_once(order, dim):
    """Expanding every multiset of [0, dim) yields each of dim**order coordinates once."""
    ms = _all_multisets(dim, order)
    total = dim ** order
    r = oracle.expand(order, dim, ms, coords_cap=total + 1)
    assert r["effective_nnz"] == total
    coords = r["coords"]
    assert coords.shape[0] == total
    keys = np.zeros(total, dtype=np.int64)
    for t in range(order):
        keys = keys * dim + coords[:, t]
    assert np.unique(keys).size == total


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_per_entry_counts_are_distinct_permutation_counts(order):
    """Per entry, the number of expanded coordinates equals the number of
    distinct arrangements of the tuple (counted with a Python set)."""
    dim = 6
    ms = _all_multisets(dim, order)
    r = oracle.expand(order, dim, ms, per_entry=True)
    for e, c in enumerate(ms):
        assert r["per_entry"][e] == len(set(itertools.permutations(c.tolist())))


def test_pattern_histogram_counts_entries():
    order, dim = 4, 6
    ms = _all_multisets(dim, order)
    r = oracle.expand(order, dim, ms)
    for mask in range(1 << (order - 1)):
        want = sum(1 for c in ms.tolist()
                   if all((c[t] == c[t + 1]) == bool(mask >> t & 1) for t in range(order - 1)))
        assert r["hist"][mask] == want
    assert r["entries"] == len(ms)


# ----------------------------------------------------------- brute force ----

def _dense_from_list(order, dim, idx, val):
    T = np.zeros((dim,) * order)
    for c, v in zip(idx.T.tolist(), val.tolist()):
        for p in set(itertools.permutations(c)):
            T[p] += v
    return T


EINSUM = {2: "ik,kr->ir", 3: "ikl,kr,lr->ir", 4: "iklm,kr,lr,mr->ir", 5: "iklmn,kr,lr,mr,nr->ir"}


@pytest.mark.parametrize("order,dim,nnz,rep", [(2, 8, 20, 0.2), (3, 8, 60, 0.5), (4, 8, 80, 0.5),
                                               (5, 8, 100, 0.6)])
def test_mttkrp_equals_dense_brute_force(order, dim, nnz, rep):
    t = synth.sym_coo(order, dim, nnz, repeat_frac=rep, seed=100 + order, R=None)
    idx = t["idx"]
    val = synth.integer_valued(idx.shape[1], seed=7)
    B = synth.integer_valued((dim, 5), seed=8)
    # every equality pattern is present
    r = oracle.expand(order, dim, idx.T)
    assert all(h > 0 for h in r["hist"]), r["hist"]
    T = _dense_from_list(order, dim, idx, val)
    want = np.einsum(EINSUM[order], T, *([B] * (order - 1)))
    C, counts = oracle.mttkrp(order, dim, idx.T, val, B)
    np.testing.assert_array_equal(C, want)
    assert counts["effective_nnz"] == np.count_nonzero(
        _dense_from_list(order, dim, idx, np.ones_like(val)))


def test_ssymv_syprd_equal_dense_brute_force():
    m = synth.ssymv_uniform(40, 5, seed=21)
    n = m["n"]
    val = synth.integer_valued(m["col"].size, seed=22)
    x = synth.integer_valued(n, seed=23)
    A = np.zeros((n, n))
    pattern = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    for i, j, v in zip(rows, m["col"], val):
        A[i, j] += v
        pattern[i, j] = True
        if i != j:
            A[j, i] += v
            pattern[j, i] = True
    y, counts = oracle.ssymv(n, m["rowptr"], m["col"], val, x)
    np.testing.assert_array_equal(y, A @ x)
    assert counts["effective_nnz"] == np.count_nonzero(pattern)
    s, sa, _ = oracle.syprd(n, m["rowptr"], m["col"], val, x)
    assert s == x @ A @ x


# ----------------------------------------------------------- closed form ----

@pytest.mark.parametrize("order,dim", [(2, 9), (3, 8), (4, 6), (5, 5)])
def test_rank_one_closed_form(order, dim):
    """T = u (x) ... (x) u  gives  C[i, r] = u_i (u . B[:, r])**(order-1)."""
    u = synth.integer_valued(dim, seed=31, low=-2, high=2)
    B = synth.integer_valued((dim, 4), seed=32, low=-2, high=2)
    ms = _all_multisets(dim, order)
    val = np.prod(u[ms], axis=1)
    C, _ = oracle.mttkrp(order, dim, ms, val, B)
    want = u[:, None] * (u @ B)[None, :] ** (order - 1)
    np.testing.assert_array_equal(C, want)


def test_rank_one_ssymv_syprd():
    """A = u u^T gives y = u (u . x) and x^T A x = (u . x)**2."""
    n = 12
    u = synth.integer_valued(n, seed=33)
    x = synth.integer_valued(n, seed=34)
    ms = _all_multisets(n, 2)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(np.bincount(ms[:, 0], minlength=n))
    val = u[ms[:, 0]] * u[ms[:, 1]]
    y, _ = oracle.ssymv(n, rowptr, ms[:, 1], val, x)
    np.testing.assert_array_equal(y, u * (u @ x))
    s, _, _ = oracle.syprd(n, rowptr, ms[:, 1], val, x)
    assert s == (u @ x) ** 2


# --------------------------------------------------------------- library ----

def test_ssymv_syprd_match_scipy():
    import scipy.sparse as sp
    m = synth.ssymv_uniform(500, 9, seed=41)
    n = m["n"]
    U = sp.csr_matrix((m["val"], m["col"], m["rowptr"]), shape=(n, n))
    A = U + U.T - sp.diags(U.diagonal())
    y, _ = oracle.ssymv(n, m["rowptr"], m["col"], m["val"], m["x"])
    ref = A @ m["x"]
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    s, sa, _ = oracle.syprd(n, m["rowptr"], m["col"], m["val"], m["x"])
    assert abs(s - m["x"] @ (A @ m["x"])) <= 1e-13 * sa


# ------------------------------------------------------------ invariance ----

@pytest.mark.parametrize("order", [3, 4, 5])
def test_order_invariance(order):
    dim = 12
    t = synth.sym_coo(order, dim, 150, repeat_frac=0.3, seed=50 + order, R=3)
    idx, B = t["idx"].T, t["B"]
    vi = synth.integer_valued(idx.shape[0], seed=9)
    Bi = synth.integer_valued(B.shape, seed=10)
    C0, k0 = oracle.mttkrp(order, dim, idx, vi, Bi)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(idx.shape[0])
    C1, k1 = oracle.mttkrp(order, dim, idx[perm], vi[perm], Bi)
    np.testing.assert_array_equal(C0, C1)
    assert k0 == k1
    # float inputs: same up to rounding order
    Cf0, _ = oracle.mttkrp(order, dim, idx, t["val"], B)
    Cf1, _ = oracle.mttkrp(order, dim, idx[perm], t["val"][perm], B)
    assert np.linalg.norm(Cf0 - Cf1) <= 1e-12 * np.linalg.norm(Cf0)


@pytest.mark.parametrize("order", [3, 4, 5])
def test_relabel_invariance(order):
    """Relabel indices by a permutation pi (re-sorting every tuple); then
    C'[pi(i)] = C[i] when B's rows are permuted the same way."""
    dim = 12
    t = synth.sym_coo(order, dim, 120, repeat_frac=0.3, seed=60 + order)
    idx = t["idx"].T
    val = synth.integer_valued(idx.shape[0], seed=1)
    B = synth.integer_valued((dim, 4), seed=2)
    pi = np.random.Generator(np.random.PCG64(3)).permutation(dim)
    idx2 = np.sort(pi[idx], axis=1).astype(np.int32)
    B2 = np.empty_like(B)
    B2[pi] = B
    C, _ = oracle.mttkrp(order, dim, idx, val, B)
    C2, _ = oracle.mttkrp(order, dim, idx2, val, B2)
    np.testing.assert_array_equal(C2[pi], C)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_mode_invariance(order):
    """Any index slot may serve as the output slot of a symmetric tensor."""
    dim = 24 if order == 2 else 12
    t = synth.sym_coo(order, dim, 100, repeat_frac=0.05 if order == 2 else 0.4, seed=70 + order)
    idx = t["idx"].T
    val = synth.integer_valued(idx.shape[0], seed=4)
    B = synth.integer_valued((dim, 3), seed=5)
    C0, _ = oracle.mttkrp(order, dim, idx, val, B, out_slot=0)
    for s in range(1, order):
        Cs, _ = oracle.mttkrp(order, dim, idx, val, B, out_slot=s)
        np.testing.assert_array_equal(Cs, C0)


def test_linearity_and_duplicates_add():
    order, dim = 4, 8
    t1 = synth.sym_coo(order, dim, 60, repeat_frac=0.3, seed=81)
    t2 = synth.sym_coo(order, dim, 50, repeat_frac=0.3, seed=82)
    v1 = synth.integer_valued(60, seed=83)
    v2 = synth.integer_valued(50, seed=84)
    B = synth.integer_valued((dim, 3), seed=85)
    C1, _ = oracle.mttkrp(order, dim, t1["idx"].T, v1, B)
    C2, _ = oracle.mttkrp(order, dim, t2["idx"].T, v2, B)
    idx = np.concatenate([t1["idx"].T, t2["idx"].T])  # may hold duplicate tuples
    C12, k = oracle.mttkrp(order, dim, idx, np.concatenate([v1, v2]), B)
    np.testing.assert_array_equal(C12, C1 + C2)
    assert k["entries"] == 110


def test_noncanonical_tuples_sorted_and_counted():
    dim = 6
    idx = np.array([[4, 1, 2], [1, 2, 4], [5, 5, 0]], dtype=np.int32)
    val = np.array([1.0, 2.0, 3.0])
    B = synth.integer_valued((dim, 2), seed=6)
    C, k = oracle.mttkrp(3, dim, idx, val, B)
    Cs, ks = oracle.mttkrp(3, dim, np.sort(idx, axis=1), val, B)
    np.testing.assert_array_equal(C, Cs)
    assert k["noncanonical"] == 2 and ks["noncanonical"] == 0


def test_row_mask_restricts_output_only():
    order, dim = 3, 10
    t = synth.sym_coo(order, dim, 80, repeat_frac=0.2, seed=90, R=4)
    mask = np.zeros(dim, dtype=np.uint8)
    mask[[1, 4, 9]] = 1
    C, k = oracle.mttkrp(order, dim, t["idx"].T, t["val"], t["B"])
    Cm, km = oracle.mttkrp(order, dim, t["idx"].T, t["val"], t["B"], row_mask=mask)
    np.testing.assert_array_equal(Cm[mask == 1], C[mask == 1])
    assert not Cm[mask == 0].any()
    assert k == km


def test_out_of_range_index_rejected():
    with pytest.raises(ValueError):
        oracle.mttkrp(3, 5, np.array([[0, 1, 5]]), [1.0], np.ones((5, 2)))


# ------------------------------------------------------------------ bf16 ----

def test_round_bf16_matches_torch_conversion():
    import torch
    rng = np.random.Generator(np.random.PCG64(5))
    x = np.concatenate([
        rng.uniform(-1, 1, 20000).astype(np.float32),
        (rng.standard_normal(20000) * 1e-30).astype(np.float32),
        (rng.standard_normal(2000) * 1e-39).astype(np.float32),   # subnormal
        np.array([0.0, -0.0, 1.0, -2.5, 3.0e38], dtype=np.float32),
    ])
    # exact ties: the low 16 bits are 0x8000
    ties = (rng.integers(0, 1 << 15, 4000).astype(np.uint32) << 16 | 0x8000) + (0x3F000000)
    x = np.concatenate([x, ties.astype(np.uint32).view(np.float32)])
    ours = oracle.round_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


# ----------------------------------------------------- all-core variants ----

@pytest.mark.parametrize("threads", [2, 3, 0])
def test_all_core_oracle_equals_single_thread(threads):
    """The all-core oracle (static partition of the stored entries, private
    FP64 outputs added in thread order) gives the single-threaded result: bit
    for bit with integer-valued inputs (every partial sum is exact), and with
    the same counts. It adds nothing of its own to the definition."""
    t = synth.sym_coo(4, 30, 4000, 0.3, seed=71)
    v = synth.integer_valued(t["val"].size, seed=72).astype(np.float64)
    B = synth.integer_valued((30, 6), seed=73)
    C1, k1 = oracle.mttkrp(4, 30, t["idx"].T, v, B)
    Ct, kt = oracle.mttkrp(4, 30, t["idx"].T, v, B, threads=threads)
    np.testing.assert_array_equal(Ct, C1)
    assert kt == k1
    m = synth.ssymv_uniform(701, 9, seed=74)
    a = synth.integer_valued(m["col"].size, seed=75).astype(np.float64)
    x = synth.integer_valued(701, seed=76).astype(np.float64)
    y1, c1 = oracle.ssymv(701, m["rowptr"], m["col"], a, x)
    yt, ct = oracle.ssymv(701, m["rowptr"], m["col"], a, x, threads=threads)
    np.testing.assert_array_equal(yt, y1)
    assert ct == c1
    # and a dense brute force for the same matrix
    A = np.zeros((701, 701))
    rows = np.repeat(np.arange(701), np.diff(m["rowptr"]))
    A[rows, m["col"]] = a
    A[m["col"], rows] = a
    np.testing.assert_array_equal(yt, A @ x)
