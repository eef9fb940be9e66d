"""GPU tests of the serving runtime: results in a concurrent mix equal the same
requests served alone and the oracle; admission blocks under a small budget
and resumes; oversize requests are rejected; requests that arrive while
others run are admitted and complete."""
import numpy as np
import pytest

import oracle
import paper_2406_09266_amd as systec
from paper_2406_09266_amd import synth

from gpu_util import dev, f32, rel_err, wide_step_matrix

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _pool():
    """A small mixed pool: two matrices and two tensors (orders 3 and 4)."""
    mats = [synth.ssymv_random_degree(30000, 12, seed=71), synth.ssymv_rmat(scale=15, batch=1 << 17,
                                                                            seed=72)]
    tens = [synth.sym_coo(3, 2000, 60000, 0.05, seed=73), synth.sym_coo(4, 500, 40000, 0.05, seed=74)]
    return mats, tens


def _register(srv, mats, tens):
    ids = []
    for m in mats:
        ids.append(srv.register(systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]),
                                                      dev(m["val"].astype(np.float32)))))
    for t in tens:
        ids.append(srv.register(systec.Tensor.from_coo([dev(a) for a in t["idx"]],
                                                      dev(t["val"].astype(np.float32)), t["dim"])))
    return ids


def _requests(mats, tens, count, seed):
    """(pool index, input as numpy, R) for `count` requests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(count):
        p = int(rng.integers(0, len(mats) + len(tens)))
        if p < len(mats):
            reqs.append((p, synth.dense_uniform(mats[p]["n"], seed=1000 + k), 1))
        else:
            t = tens[p - len(mats)]
            R = int(rng.choice([8, 16, 32]))
            reqs.append((p, synth.dense_uniform((t["dim"], R), seed=1000 + k), R))
    return reqs


def _submit(srv, ids, mats, tens, req, bf16):
    """Submits without synchronizing: the request is ordered after the
    current stream, which wrote its input."""
    import torch
    p, inp, R = req
    x = dev(inp.astype(np.float32))
    if bf16:
        x = systec.quantize_bf16(x)
    if p < len(mats):
        out = torch.empty(mats[p]["n"], device="cuda")
    else:
        out = torch.empty((tens[p - len(mats)]["dim"], R), device="cuda")
    return srv.submit(ids[p], x, out), out


def _oracle(mats, tens, req, bf16):
    p, inp, R = req
    ref = oracle.round_bf16(inp.astype(np.float32)) if bf16 else f32(inp)
    if p < len(mats):
        m = mats[p]
        return oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]), ref)[0]
    t = tens[p - len(mats)]
    return oracle.mttkrp(t["order"], t["dim"], t["idx"].T, f32(t["val"]), ref)[0]


@pytest.mark.parametrize("bf16,streams,inflight", [(False, 0, 0), (True, 0, 0), (True, 1, 1),
                                                    (True, 1, 3)])
def test_mix_equals_alone_and_oracle(bf16, streams, inflight):
    mats, tens = _pool()
    reqs = _requests(mats, tens, 24, seed=5)
    with systec.Server(budget_bytes=8 << 30, max_slots=8, step_work_nnz=1 << 17,
                       streams=streams, max_inflight=inflight) as srv:
        ids = _register(srv, mats, tens)
        # alone: one request at a time
        alone = []
        for r in reqs:
            rid, out = _submit(srv, ids, mats, tens, r, bf16)
            srv.wait(rid, 60_000_000)
            alone.append(out.cpu().numpy())
        # mix: all at once (small step budget: requests share steps)
        outs = []
        for r in reqs:
            outs.append(_submit(srv, ids, mats, tens, r, bf16))
        for rid, _ in outs:
            srv.wait(rid, 60_000_000)
        st = srv.stats()
    for r, a, (_, o) in zip(reqs, alone, outs):
        mix = o.cpu().numpy()
        assert rel_err(mix, a) <= TOL32
        assert rel_err(mix, _oracle(mats, tens, r, bf16)) <= TOL32
    assert st["completed"] == 48 and st["failed"] == 0
    assert st["p99_us"] >= st["p50_us"] > 0


@pytest.mark.parametrize("bf16,step_work", [(False, 1 << 14), (True, 1 << 14), (True, 1 << 26)])
def test_relabeled_matrices_are_served(bf16, step_work):
    """Matrices stored with their vertices ordered by degree, served next to a
    tensor: requests that span several steps (small step budget) and requests
    that finish in one step both give the oracle's result."""
    mats = [synth.ssymv_rmat(scale=14, batch=1 << 16, seed=91),
            synth.ssymv_random_degree(20000, 10, seed=92)]
    tens = [synth.sym_coo(3, 1500, 40000, 0.05, seed=93)]
    reqs = _requests(mats, tens, 16, seed=17)
    with systec.Server(budget_bytes=8 << 30, max_slots=6, step_work_nnz=step_work) as srv:
        ids = [srv.register(systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]),
                                                   dev(m["val"].astype(np.float32)), relabel=True))
               for m in mats]
        ids += _register(srv, [], tens)
        outs = [_submit(srv, ids, mats, tens, r, bf16) for r in reqs]
        for rid, _ in outs:
            srv.wait(rid, 60_000_000)
        st = srv.stats()
    for r, (_, o) in zip(reqs, outs):
        assert rel_err(o.cpu().numpy(), _oracle(mats, tens, r, bf16)) <= TOL32
    assert st["completed"] == 16 and st["failed"] == 0


@pytest.mark.parametrize("relabel", [False, True])
def test_wide_steps_are_served(relabel):
    """A matrix with steps whose columns overflow the packed offsets (the
    kernels read those steps' columns unpacked), served in FP32 and BF16."""
    m = wide_step_matrix()
    reqs = [(0, synth.dense_uniform(m["n"], seed=2000 + k), 1) for k in range(4)]
    with systec.Server(budget_bytes=8 << 30, max_slots=4, step_work_nnz=1 << 14) as srv:
        ids = [srv.register(systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]),
                                                   dev(m["val"].astype(np.float32)),
                                                   relabel=relabel))]
        outs = [(_submit(srv, ids, [m], [], r, k % 2 == 1), k % 2 == 1)
                for k, r in enumerate(reqs)]
        for (rid, _), _ in outs:
            srv.wait(rid, 60_000_000)
    for r, ((_, o), bf16) in zip(reqs, outs):
        assert rel_err(o.cpu().numpy(), _oracle([m], [], r, bf16)) <= TOL32


def test_relabeled_request_counts_its_scratch():
    """A request on a relabeled matrix holds its input and output twice (the
    copies in the stored order): a budget with room for one plain request
    next to the matrix rejects it."""
    import torch
    m = synth.ssymv_rmat(scale=13, batch=1 << 15, seed=95)

    def tensor():
        return systec.Tensor.from_csr(dev(m["rowptr"]), dev(m["col"]),
                                      dev(m["val"].astype(np.float32)), relabel=True)
    with systec.Server(budget_bytes=1 << 40) as probe:
        probe.register(tensor())
        resident = probe.stats()["bytes_in_use"]
    one = m["n"] * (4 + 4)
    x = dev(synth.dense_uniform(m["n"], seed=96).astype(np.float32))
    y = torch.empty(m["n"], device="cuda")
    torch.cuda.synchronize()
    with systec.Server(budget_bytes=resident + one + one // 2) as srv:
        tid = srv.register(tensor())
        with pytest.raises(systec.SystecError) as e:
            srv.submit(tid, x, y)
        assert e.value.status_name == "SYSTEC_EBUDGET"
    with systec.Server(budget_bytes=resident + 2 * one + one // 4) as srv:
        tid = srv.register(tensor())
        srv.wait(srv.submit(tid, x, y), 60_000_000)
    want = oracle.ssymv(m["n"], m["rowptr"], m["col"], f32(m["val"]),
                        synth.dense_uniform(m["n"], seed=96).astype(np.float32).astype(np.float64))[0]
    assert rel_err(y.cpu().numpy(), want) <= TOL32


def test_small_budget_blocks_and_resumes():
    import torch
    m = synth.ssymv_random_degree(200000, 16, seed=81)
    mats = [m]
    with systec.Server(budget_bytes=1 << 40, max_slots=4) as probe:
        _register(probe, mats, [])
        resident = probe.stats()["bytes_in_use"]
    one = m["n"] * (4 + 4)  # one FP32 request: input + output
    reqs = _requests(mats, [], 20, seed=9)
    xs = [dev(r[1].astype(np.float32)) for r in reqs]
    ys = [torch.empty(m["n"], device="cuda") for _ in reqs]
    torch.cuda.synchronize()
    # room for the tensor and one request at a time
    with systec.Server(budget_bytes=resident + one + one // 2, max_slots=4,
                       step_work_nnz=1 << 14) as srv:
        ids = _register(srv, mats, [])
        rids = [srv.submit(ids[0], x, y) for x, y in zip(xs, ys)]
        states = [srv.poll(rid) for rid in rids]
        assert states.count(srv.RUNNING) <= 1
        assert srv.QUEUED in states  # the budget holds later requests back
        for rid in rids:
            srv.wait(rid, 60_000_000)
        assert srv.stats()["completed"] == 20
    for r, y in zip(reqs, ys):
        assert rel_err(y.cpu().numpy(), _oracle(mats, [], r, False)) <= TOL32
    # a request that can never fit next to the resident tensor is rejected
    with systec.Server(budget_bytes=resident + one // 2, max_slots=4) as srv:
        ids = _register(srv, mats, [])
        with pytest.raises(systec.SystecError) as e:
            srv.submit(ids[0], xs[0], ys[0])
        assert e.value.status_name == "SYSTEC_EBUDGET"
        assert srv.stats()["rejected"] == 1


def test_arrivals_while_running_are_admitted():
    """A long request runs; requests that arrive while it is on the GPU are
    admitted into its steps and finish before it (each step gives every
    running request at least one work unit); every result matches the same
    request computed alone."""
    import time
    import torch
    mats, tens = _pool()
    reqs = _requests(mats, tens, 20, seed=11)
    big = synth.gpu_sym_coo(3, 100_000, 20_000_000, 0.01, seed=12)
    B = systec.quantize_bf16(torch.rand((100_000, 8), device="cuda") * 2 - 1)
    alone = systec.Tensor.from_coo(big["idx"], big["val"], 100_000).mttkrp(B)
    torch.cuda.synchronize()
    with systec.Server(budget_bytes=16 << 30, max_slots=32, step_work_nnz=1) as srv:
        ids = _register(srv, mats, tens)
        bid = srv.register(systec.Tensor.from_coo(big["idx"], big["val"], 100_000))
        del big
        out_big = torch.empty((100_000, 8), device="cuda")
        torch.cuda.synchronize()
        rid_big = srv.submit(bid, B, out_big)
        t0 = time.time()
        while srv.poll(rid_big) == srv.QUEUED and time.time() - t0 < 30:
            time.sleep(1e-4)
        assert srv.poll(rid_big) == srv.RUNNING
        outs = [_submit(srv, ids, mats, tens, r, True) for r in reqs]
        done_while_big_ran = 0
        while srv.poll(rid_big) == srv.RUNNING and time.time() - t0 < 60:
            done_while_big_ran = sum(srv.poll(rid) == srv.DONE for rid, _ in outs)
            time.sleep(2e-4)
        for rid, _ in outs:
            srv.wait(rid, 60_000_000)
        srv.wait(rid_big, 60_000_000)
        st = srv.stats()
    assert done_while_big_ran >= 1
    assert st["completed"] == 21 and st["steps"] >= 2
    assert rel_err(out_big.cpu().numpy(), alone.cpu().numpy()) <= TOL32
    for r, (_, o) in zip(reqs, outs):
        assert rel_err(o.cpu().numpy(), _oracle(mats, tens, r, True)) <= TOL32


def test_unknown_ids_and_timeout():
    with systec.Server(budget_bytes=1 << 30) as srv:
        with pytest.raises(systec.SystecError) as e:
            srv.poll(12345)
        assert e.value.status_name == "SYSTEC_ENOTFOUND"
        with pytest.raises(systec.SystecError) as e:
            srv.wait(12345, 10)
        assert e.value.status_name == "SYSTEC_ENOTFOUND"


def test_submit_waits_for_the_callers_stream():
    """A request submitted right after slow work on the caller's stream that
    writes its input and last uses its output buffer: the server's stream
    waits for that work (no host synchronization in between)."""
    import torch
    mats, tens = _pool()
    reqs = _requests(mats, tens, 6, seed=9)
    big = torch.rand((4096, 4096), device="cuda")
    with systec.Server(budget_bytes=8 << 30, max_slots=8, step_work_nnz=1 << 17) as srv:
        ids = _register(srv, mats, tens)
        torch.cuda.synchronize()
        outs = []
        for p, inp, R in reqs:
            src = dev(inp.astype(np.float32))
            torch.cuda.synchronize()
            x = torch.empty_like(src)
            out = torch.full((mats[p]["n"],) if p < len(mats) else (tens[p - len(mats)]["dim"], R),
                             7.0, device="cuda")
            for _ in range(8):  # slow work queued ahead of the input's write
                big = torch.mm(big, big).clamp_(-1.0, 1.0)
            out.fill_(3.0)  # the output buffer's last earlier use
            x.copy_(src)
            outs.append((srv.submit(ids[p], x, out), out, x))
        for rid, _, _ in outs:
            srv.wait(rid, 60_000_000)
    for r, (_, o, _) in zip(reqs, outs):
        assert rel_err(o.cpu().numpy(), _oracle(mats, tens, r, False)) <= TOL32
