"""GPU parity of one symmetric CP-ALS step around MTTKRP against the FP64
oracle's cp_step (its MTTKRP over the expanded tensor, then dense FP64 linear
algebra in numpy).

Tolerances: the MTTKRP C element by element (1e-5 of each element's scale,
as in the MTTKRP parity tests); G = B^T B element by element (1e-5 of
(|B|^T |B|)); B_new = C (G^(N-1))^-1 normwise 1e-5 (the inputs here give
G^(N-1) a condition number near 1, so the FP32 Cholesky solve adds error of
the order of FP32 rounding); the four fit scalars within 1e-5 of the sum of
the magnitudes of their terms (they can cancel). BF16 factors: the same
against the oracle on the BF16-rounded factor, and 2e-2 end to end."""
import numpy as np
import pytest

import oracle
import paper_2406_09266_amd as systec
from paper_2406_09266_amd import synth

from gpu_util import assert_elementwise, dev, f32, rel_err

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("order,dim,nnz", [(3, 300, 20011), (4, 120, 15013), (5, 60, 9001),
                                           (3, 20000, 200003)])
@pytest.mark.parametrize("R", [1, 8, 16, 32])
@pytest.mark.parametrize("bdtype", ["f32", "bf16"])
def test_cp_step_matches_oracle(order, dim, nnz, R, bdtype):
    t = synth.sym_coo(order, dim, nnz, repeat_frac=0.2, seed=700 + order * 11 + R)
    B = synth.dense_uniform((dim, R), seed=800 + R)
    print(f"cp step order={order} dim={dim} nnz={nnz} R={R} B={bdtype}", flush=True)
    Bd = dev(B.astype(np.float32))
    if bdtype == "bf16":
        Bd = systec.quantize_bf16(Bd)
        Bref = oracle.round_bf16(B.astype(np.float32))
    else:
        Bref = f32(B)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), dim)
    B_new, C, G, fit = T.cp_step(Bd)
    B_new, C, G, fit = (B_new.cpu().numpy(), C.cpu().numpy(), G.cpu().numpy(), fit.cpu().numpy())
    v32 = f32(t["val"])
    ref = oracle.cp_step(order, dim, t["idx"].T, v32, Bref)
    # the MTTKRP and the Gram matrix, element by element
    scaleC, _ = oracle.mttkrp(order, dim, t["idx"].T, np.abs(v32), np.abs(Bref))
    assert_elementwise(C, ref["C"], scaleC, TOL32, "cp step C")
    assert_elementwise(G, ref["G"], np.abs(Bref).T @ np.abs(Bref), TOL32, "cp step G")
    # the update, normwise
    assert rel_err(B_new, ref["B_new"]) <= TOL32
    # the fit scalars against the magnitudes of their terms
    absG = np.abs(ref["G"])
    s_inner = float(np.sum(np.abs(ref["C"]) * np.abs(Bref)))
    s_model = float(np.sum(absG ** order))
    scales = [ref["norm_T2"], s_inner, s_model, ref["norm_T2"] + 2 * s_inner + s_model]
    for got, want, sc, name in zip(fit, (ref["norm_T2"], ref["inner"], ref["norm_M2"],
                                         ref["resid2"]), scales,
                                   ("norm_T2", "inner", "norm_M2", "resid2")):
        assert abs(got - want) <= TOL32 * sc, (name, got, want, sc)
    if bdtype == "bf16":  # end to end against the unrounded factor
        e2e = oracle.cp_step(order, dim, t["idx"].T, t["val"], B)
        assert rel_err(B_new, e2e["B_new"]) <= 2e-2
    T.close()


@pytest.mark.parametrize("order", [3, 4, 5])
def test_cp_step_rank_one_closed_form(order):
    """T = u (x) ... (x) u over every multiset of [0, I): with R = 1,
    C = u (u . b)^(N-1), G = b . b and B_new = u ((u . b) / (b . b))^(N-1)."""
    import itertools
    I = {3: 30, 4: 14, 5: 9}[order]
    u = synth.integer_valued(I, seed=3).astype(np.float64)
    u[u == 0] = 1.0
    tuples = np.array(list(itertools.combinations_with_replacement(range(I), order)), np.int32)
    vals = np.prod(u[tuples], axis=1)
    b = synth.dense_uniform((I, 1), seed=4)
    b32 = f32(b)
    T = systec.Tensor.from_coo([dev(np.ascontiguousarray(tuples[:, k])) for k in range(order)],
                               dev(vals.astype(np.float32)), I)
    B_new, C, G, fit = (x.cpu().numpy() for x in T.cp_step(dev(b.astype(np.float32))))
    ub = float(u @ b32[:, 0])
    bb = float(b32[:, 0] @ b32[:, 0])
    # (u . b) sums terms of both signs: each result is held to 1e-5 of the
    # same closed form on magnitudes, |u| (|u| . |b|)^(N-1)
    aub = float(np.abs(u) @ np.abs(b32[:, 0]))
    scale = np.abs(u) * aub ** (order - 1)
    assert np.all(np.abs(C[:, 0] - u * ub ** (order - 1)) <= TOL32 * scale)
    assert abs(G[0, 0] - bb) <= TOL32 * bb
    assert np.all(np.abs(B_new[:, 0] - u * (ub / bb) ** (order - 1))
                  <= TOL32 * scale / bb ** (order - 1))
    # ||T||^2 = (u.u)^N, <T,[[b]]> = (u.b)^N, ||[[b]]||^2 = (b.b)^N
    uu = float(u @ u)
    for got, want, sc in zip(fit[:3], (uu ** order, ub ** order, bb ** order),
                             (uu ** order, aub ** order, bb ** order)):
        assert abs(got - want) <= TOL32 * sc


def test_cp_step_rejects_bad_arguments():
    t = synth.sym_coo(3, 50, 1000, 0.0, seed=5)
    T = systec.Tensor.from_coo([dev(a) for a in t["idx"]], dev(t["val"].astype(np.float32)), 50)
    with pytest.raises(systec.SystecError) as e:
        T.cp_step(dev(synth.dense_uniform((50, 65), seed=6).astype(np.float32)))
    assert e.value.status_name == "SYSTEC_EINVAL"
    A = systec.Tensor.from_csr(dev(np.array([0, 1], np.int32)), dev(np.array([0], np.int32)),
                               dev(np.array([1.0], np.float32)))
    with pytest.raises((systec.SystecError, ValueError)):
        A.cp_step(dev(np.ones((1, 4), np.float32)))
