"""The host symmetric loops (the benchmark's CPU analog of the paper's
symmetric loop) against the oracle's expanded definitions: SSYMV over the
stored triangle and MTTKRP over canonical tuples give the oracle's result on
tensors holding every composition of repeated indices."""
import numpy as np
import pytest

import oracle
from oracle import host_loops
from paper_2406_09266_amd import synth


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("case", ["uniform", "rmat", "diagonal"])
def test_host_ssymv_equals_oracle(case):
    m = {"uniform": lambda: synth.ssymv_uniform(3001, 7, seed=61),
         "rmat": lambda: synth.ssymv_rmat(scale=12, batch=1 << 14, seed=62),
         "diagonal": lambda: synth.ssymv_uniform(500, 0, seed=63)}[case]()
    y = host_loops.ssymv(m["n"], m["rowptr"], m["col"], m["val"], m["x"])
    want, _ = oracle.ssymv(m["n"], m["rowptr"], m["col"], m["val"], m["x"])
    assert _rel(y, want) <= 1e-13


@pytest.mark.parametrize("order,dim,repeat", [(3, 40, 0.2), (4, 25, 0.5), (5, 14, 0.5)])
def test_host_mttkrp_equals_oracle(order, dim, repeat):
    t = synth.sym_coo(order, dim, 3000, repeat_frac=repeat, seed=70 + order)
    B = synth.dense_uniform((dim, 6), seed=71)
    C = host_loops.mttkrp(order, dim, t["idx"].T, t["val"], B)
    want, counts = oracle.mttkrp(order, dim, t["idx"].T, t["val"], B)
    assert all(h > 0 for h in counts["hist"])  # every composition present
    assert _rel(C, want) <= 1e-13


def test_host_loops_reject_bad_indices():
    with pytest.raises(ValueError):
        host_loops.ssymv(3, np.array([0, 1, 1, 1]), np.array([5]), np.array([1.0]), np.ones(3))
    with pytest.raises(ValueError):  # a tuple not in ascending order
        host_loops.mttkrp(3, 4, np.array([[2, 1, 3]]), np.array([1.0]), np.ones((4, 2)))
