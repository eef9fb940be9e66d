#!/usr/bin/env python3
"""Benchmark: symmetric sparse SSYMV / MTTKRP on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--form f32|bf16]

A step is one library call of the hot path over one batch of synthetic
input: output zeroing plus the symmetric kernel over the canonical entries.
Inputs are resident in HBM before the timed region starts. The metric is
effective nnz/s: the number of entries of the fully expanded (non-symmetric)
tensor, sum over stored entries of N!/prod(m!), divided by the time of a
step. The headline workload (default: the R-MAT SSYMV) fills the top level of
the one JSON line; every workload named by --also (default: the 3-D and 5-D
MTTKRP) is measured in the same run and reported in a record of its own with
the same fields. Each record carries:
  value, ms_per_step   warm steps, the K timed ones
  cold                 min/median of single calls after a 512 MiB cache flush
  roofline             algorithmic bytes / the dominant kernel's own time
                       (HIP events around its launches, on its stream), as a
                       fraction of the 8 TB/s peak and of a measured device
                       copy; traffic from the committed rocprofv3 counters
  nonsymmetric         the same call on the expanded operand
  oracle_rel_err       against the FP64 oracle on the values the GPU saw
  e2e_rel_err          against the FP64 oracle on the original FP64 inputs
  cpu_baseline         the oracle on every host core (its all-core variant),
  cpu_baseline_1core   and on one core
  cpu_symmetric_loop_1core  the method's own loop over the canonical entries
                       on one host core, with its speedup over the oracle's
                       expanded loop (the host analog of the paper's
                       symmetric-against-naive comparison)

Workloads (synthetic, seeded; shaped like the paper's):
  ssymv_rmat   (default) R-MAT scale 22, n=4,194,304, avg degree 16, upper CSR
  ssymv_small  n=2,000, ~10 stored entries per row
  mttkrp3      order 3, I=100,000, 20M canonical entries, R=32
  mttkrp5      order 5, I=5,000, 5M canonical entries, R=16
  served_mix   Poisson arrivals against resident tensors (its own JSON line)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ssymv_rmat",
                    choices=["ssymv_rmat", "ssymv_small", "mttkrp3", "mttkrp5", "served_mix"])
    ap.add_argument("--pool-per-kind", type=int, default=8,
                    help="served_mix: resident tensors per kind (SSYMV, 3-D, 4-D)")
    ap.add_argument("--requests", type=int, default=1000,
                    help="served_mix: requests per Poisson run")
    ap.add_argument("--step-work", type=int, default=1 << 27,
                    help="served_mix: stored entries per serving step")
    ap.add_argument("--max-slots", type=int, default=32,
                    help="served_mix: requests running at once")
    ap.add_argument("--max-inflight", type=int, default=0,
                    help="served_mix: steps queued on the device at once (0: the server default)")
    ap.add_argument("--relabel", default="auto", choices=["auto", "on", "off"],
                    help="SSYMV: prepare the matrix with its vertices ordered by degree "
                         "(auto: when the degrees are skewed)")
    ap.add_argument("--served-dtype", default="bf16", choices=["bf16", "f32"],
                    help="served_mix: input dtype of the served requests (the plain form is FP32)")
    ap.add_argument("--min-step-work", type=int, default=0,
                    help="served_mix: step budget with one running request (0: fixed steps)")
    ap.add_argument("--streams", type=int, default=0,
                    help="served_mix: 1 runs a step's kernel kinds in order on one stream, "
                         "0 one stream per kind")
    ap.add_argument("--loads", default="0.5,0.8,0.95",
                    help="served_mix: offered loads as fractions of saturation")
    ap.add_argument("--algo", default="auto", choices=["auto", "views", "atomic", "lds"],
                    help="MTTKRP: how non-leading-slot updates are resolved (auto: the "
                         "library's choice for the shape)")
    ap.add_argument("--form", default="bf16", choices=["f32", "bf16"],
                    help="storage of x / B (arithmetic is FP32 either way)")
    ap.add_argument("--path", default="prepared", choices=["prepared", "oneshot"],
                    help="prepared: the operand rearranged once (panel format / slot "
                         "views; setup untimed, as the paper leaves data rearrangement out "
                         "of its timings); oneshot: the canonical CSR/COO as given")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--also", default="mttkrp3,mttkrp5",
                    help="further workloads measured in the same run, each reported in a "
                         "record of its own in the same JSON line ('' for none)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the non-symmetric comparison kernel")
    ap.add_argument("--only-step", action="store_true",
                    help="time the step alone (no cold runs, other paths, comparisons or "
                         "errors): for profiler runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (scales the "
                         "HBM byte counters of a rocprofv3 --pmc run)")
    return ap.parse_args()


def src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2406_09266_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key, current_hash, launches_bytes):
    """HBM traffic per launch from the committed rocprofv3 PMC summary, or None
    if there is none for this kernel or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f).get(kernel_key)
    if not d or d.get("source_hash") != current_hash:
        return None
    return d.get("bytes_per_launch")


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def degree_ordered_csr(torch, rp, col, val, perm):
    """Upper-triangle CSR of P A P^T for perm (position -> caller's vertex), on
    the device: the comparison kernels then see the order the symmetric path
    stores its matrix in (setup, not timed)."""
    n = rp.numel() - 1
    dev = rp.device
    inv = torch.empty(n, dtype=torch.int64, device=dev)
    inv[perm.long()] = torch.arange(n, dtype=torch.int64, device=dev)
    rows = torch.repeat_interleave(torch.arange(n, dtype=torch.int64, device=dev),
                                   (rp[1:] - rp[:-1]).long())
    r2, c2 = inv[rows], inv[col.long()]
    del rows
    lo, hi = torch.minimum(r2, c2), torch.maximum(r2, c2)
    key, order = torch.sort(lo * n + hi)
    del lo, hi, r2, c2
    lo, hi = key // n, key % n
    rp2 = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rp2[1:] = torch.cumsum(torch.bincount(lo, minlength=n), 0)
    return rp2.int(), hi.int(), val[order].contiguous()


def rocsparse_spmv(torch, rp, col, val, x, steps, warmup):
    """rocSPARSE general CSR SpMV (adaptive algorithm, FP32) on a full matrix:
    an outside reference point for the comparison, not part of the library.
    Returns (seconds per call, y)."""
    import ctypes
    from ctypes import byref, c_float, c_int, c_int64, c_size_t, c_void_p
    L = ctypes.CDLL(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocsparse.so"))
    n, nnz = rp.numel() - 1, col.numel()
    I32, F32, OP_NONE, ADAPTIVE = 2, 151, 111, 2
    P = lambda t: c_void_p(t.data_ptr())  # noqa: E731

    def ok(st, what):
        if st != 0:
            raise RuntimeError(f"rocsparse {what}: status {st}")

    h, mat, xv, yv = c_void_p(), c_void_p(), c_void_p(), c_void_p()
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    ok(L.rocsparse_create_handle(byref(h)), "create_handle")
    try:
        ok(L.rocsparse_set_stream(h, c_void_p(torch.cuda.current_stream().cuda_stream)), "set_stream")
        ok(L.rocsparse_create_csr_descr(byref(mat), c_int64(n), c_int64(n), c_int64(nnz), P(rp), P(col),
                                        P(val), c_int(I32), c_int(I32), c_int(0), c_int(F32)), "csr descr")
        ok(L.rocsparse_create_dnvec_descr(byref(xv), c_int64(n), P(x), c_int(F32)), "x descr")
        ok(L.rocsparse_create_dnvec_descr(byref(yv), c_int64(n), P(y), c_int(F32)), "y descr")
        alpha, beta, size = c_float(1.0), c_float(0.0), c_size_t(0)

        def call(stage, buf):
            return L.rocsparse_spmv(h, c_int(OP_NONE), byref(alpha), mat, xv, byref(beta), yv,
                                    c_int(F32), c_int(ADAPTIVE), c_int(stage), byref(size), buf)
        ok(call(1, None), "buffer size")
        buf = torch.empty(max(1, size.value), dtype=torch.uint8, device=x.device)
        ok(call(2, P(buf)), "preprocess")
        ok(call(3, P(buf)), "compute")
        sec = timed(lambda: call(3, P(buf)), steps, warmup)
        torch.cuda.synchronize()
        return sec, y
    finally:
        for v in (xv, yv):
            if v.value:
                L.rocsparse_destroy_dnvec_descr(v)
        if mat.value:
            L.rocsparse_destroy_spmat_descr(mat)
        L.rocsparse_destroy_handle(h)


def kernel_ms(fn, reps):
    """Average duration of the library's hot-kernel launches inside fn()."""
    import paper_2406_09266_amd as systec
    import torch
    torch.cuda.synchronize()
    with systec.KernelTimer() as kt:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    return kt.total_ms / max(1, kt.launches), kt.launches


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cold_ms(torch, fn, reps, flush):
    """Times `reps` calls one by one with events on the current stream, each
    after a write of `flush` (512 MiB, twice the last-level cache) that is not
    timed. Returns min and median in ms."""
    torch.cuda.synchronize()
    evs = []
    for _ in range(reps):
        flush.fill_(0.0)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        evs.append((s, e))
    torch.cuda.synchronize()
    ts = sorted(s.elapsed_time(e) for s, e in evs)
    return {"ms_min": ts[0], "ms_median": ts[len(ts) // 2], "reps": reps,
            "flush_bytes": flush.numel() * 4}


def copy_ceiling_gbs(torch, dev):
    """Read + write bandwidth of a plain 1 GiB device copy (the measured
    streaming ceiling beside the 8 TB/s peak)."""
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(5):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * src.numel() * 4 / (s.elapsed_time(e) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def rel(got, want):
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def roofline(b_alg, k_ms, kernel_key, kernel_src, traffic_key, copy_gbs):
    achieved = b_alg / (k_ms * 1e-3) / 1e9
    h = src_hash(*kernel_src)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(traffic_key, h, b_alg),
            "kernel": kernel_key, "kernel_ms": k_ms, "kernel_source_hash": h,
            "copy_ceiling_gbs": copy_gbs,
            "frac_of_copy_ceiling": round(achieved / copy_gbs, 4) if copy_gbs else None}


def measure_ssymv(a, torch, systec, w, dev, flush, copy_gbs, with_cpu):
    """The SSYMV workload: the prepared call (the step), its kernel, cold
    times, the one-shot call, the stored-order call, SYPRD, the non-symmetric
    comparisons, the errors against the oracle and the oracle's own time."""
    n, U = w["n"], w["col"].size
    rp = torch.from_numpy(w["rowptr"]).to(dev)
    col = torch.from_numpy(w["col"]).to(dev)
    val = torch.from_numpy(w["val"].astype(np.float32)).to(dev)
    x32 = torch.from_numpy(w["x"].astype(np.float32)).to(dev)
    x = systec.quantize_bf16(x32) if a.form == "bf16" else x32
    y = torch.empty(n, dtype=torch.float32, device=dev)
    rows = torch.repeat_interleave(torch.arange(n, dtype=torch.int32, device=dev), rp[1:] - rp[:-1])
    hist, eff = systec.expansion_stats([rows, col], n)
    del rows
    sx = 2 if a.form == "bf16" else 4
    b_alg = 4 * (n + 1) + 8 * U + n * sx + 4 * n
    t_prep = time.perf_counter()
    relabel = {"auto": None, "on": True, "off": False}[a.relabel]
    A = systec.Tensor.from_csr(rp, col, val, relabel=relabel)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t_prep
    prepared = lambda: A.ssymv(x, out=y)  # noqa: E731
    oneshot = lambda: systec.ssymv(rp, col, val, x, out=y)  # noqa: E731
    step, other = (prepared, oneshot) if a.path == "prepared" else (oneshot, prepared)
    kernel_key = "ssymv_panel" if a.path == "prepared" else "ssymv"
    kernel_src = ("ssymv.hip", "panel_device.h", "wave_ops.h", "plan.hip")
    rec = {"config": {"workload": a.workload, "n": n, "stored_nnz": U, "effective_nnz": eff,
                      "diagonal_nnz": hist[1], "x_storage": a.form, "accumulate": "f32",
                      "vertex_order": a.relabel, "relabeled": A.vertex_order() is not None,
                      "path": a.path, "B_alg_bytes": b_alg}}
    _progress("ssymv: timed region")
    sec = timed(step, a.steps, a.warmup)
    rec["value"] = eff / sec
    rec["ms_per_step"] = sec * 1e3
    rec["config"]["canonical_nnz_per_s"] = U / sec
    k_ms, _ = kernel_ms(step, max(10, a.steps))
    rec["roofline"] = roofline(b_alg, k_ms, kernel_key, kernel_src,
                               f"{kernel_key}:{a.workload}:{a.form}", copy_gbs)
    if a.only_step:
        A.close()
        return rec
    rec["cold"] = cold_ms(torch, step, 20, flush)
    osec = timed(other, max(5, a.steps // 4), 2)
    rec["other_path"] = {"path": "oneshot" if a.path == "prepared" else "prepared",
                         "ms_per_step": osec * 1e3, "effective_nnz_per_s": eff / osec}
    perm = A.vertex_order()
    if perm is not None and a.path == "prepared":
        xs = x[perm.long()].contiguous()
        ys = torch.empty_like(y)
        tsec = timed(lambda: A.ssymv(xs, out=ys, stored_order=True), a.steps, a.warmup)
        rec["stored_order_call"] = {"ms_per_step": tsec * 1e3, "effective_nnz_per_s": eff / tsec,
                                    "vectors": "in the stored vertex order (no permutations)"}
        del xs, ys
    # the scalar form s = x^T A x (no scattered writes)
    sp = torch.empty(1, dtype=torch.float64, device=dev)
    s_alg = 4 * (n + 1) + 8 * U + n * sx
    rec["syprd"] = {"B_alg_bytes": s_alg}
    for name, fn in (("prepared", lambda: A.syprd(x, out=sp)),
                     ("oneshot", lambda: systec.syprd(rp, col, val, x, out=sp))):
        ssec = timed(fn, a.steps, a.warmup)
        rec["syprd"][name] = {"ms_per_step": ssec * 1e3, "effective_nnz_per_s": eff / ssec,
                              "hbm_frac_alg": round(s_alg / ssec / 1e9 / HBM_PEAK_GBS, 4)}
    if not a.no_compare:
        _progress("ssymv: non-symmetric comparison")
        try:
            orders = {"vertex": (rp, col, val, x)}
            if perm is not None:
                rp2, col2, val2 = degree_ordered_csr(torch, rp, col, val, perm)
                orders["degree"] = (rp2, col2, val2, x[perm.long()].contiguous())
            same = "degree" if perm is not None else "vertex"
            yf = torch.empty_like(y)
            forms, full = {}, {}
            for name, (r_, c_, v_, x_) in orders.items():
                full[name] = systec.expand_csr(r_, c_, v_) + (x_,)
                frp, fcol, fval, xo = full[name]
                forms[name] = timed(lambda: systec.spmv_csr(frp, fcol, fval, xo, out=yf),  # noqa: E731
                                    a.steps, a.warmup)
            csec = forms[same]
            rec["nonsymmetric"] = {"ms_per_step": csec * 1e3, "effective_nnz_per_s": eff / csec,
                                   "speedup_symmetric": csec / sec, "vertex_order": same,
                                   "ms_by_vertex_order": {k: v * 1e3 for k, v in forms.items()}}
            try:
                rs = {}
                for name, (frp, fcol, fval, xo) in full.items():
                    rs[name], _ = rocsparse_spmv(torch, frp, fcol, fval, xo.float(), a.steps, a.warmup)
                rec["rocsparse_general_spmv"] = {
                    "alg": "adaptive", "x_dtype": "f32",
                    "ms_by_vertex_order": {k: v * 1e3 for k, v in rs.items()},
                    "speedup_symmetric_vs_best": min(rs.values()) / sec}
            except Exception as e:  # report, do not hide
                rec["rocsparse_general_spmv"] = {"error": str(e)}
            del full, orders
        except Exception as e:  # report, do not hide
            rec["nonsymmetric"] = {"error": str(e)}
    # errors of the timed call's result against the oracle: on the values
    # the GPU saw (kernel check) and on the original FP64 inputs (end to end)
    import oracle
    step()
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    xref = x.to(torch.float64).cpu().numpy()
    vref = w["val"].astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    want, _ = oracle.ssymv(n, w["rowptr"], w["col"], vref, xref, threads=0)
    t_all = time.perf_counter() - t0
    e2e, _ = oracle.ssymv(n, w["rowptr"], w["col"], w["val"], w["x"], threads=0)
    rec["oracle_rel_err"] = rel(got, want)
    rec["e2e_rel_err"] = rel(got, e2e)
    if with_cpu:
        rec.update(cpu_legs(lambda th: oracle.ssymv(n, w["rowptr"], w["col"], vref, xref,
                                                    threads=th),
                            eff, a.cpu_seconds, t_all, "the whole workload"))
        # the method's own loop over the stored triangle on one core: the
        # host analog of the paper's symmetric-against-naive comparison
        from oracle import host_loops
        reps, t = 0, 0.0
        while (t < a.cpu_seconds / 4 and reps < 20) or reps == 0:
            t0 = time.perf_counter()
            host_loops.ssymv(n, w["rowptr"], w["col"], vref, xref)
            t += time.perf_counter() - t0
            reps += 1
        v = eff * reps / t
        rec["cpu_symmetric_loop_1core"] = {
            "value": v, "unit": "effective nnz/s", "cores": 1, "kind": "host symmetric loop",
            "sample": f"the whole workload, {reps} call(s), {t:.1f} s",
            "speedup_vs_expanded_1core": v / rec["cpu_baseline_1core"]["value"]}
    rec["setup_s"] = {"prepare_operand": round(t_prep, 3)}
    A.close()
    return rec


def cpu_legs(call, work, seconds, t_first, what):
    """The oracle timed on this host: every core (its all-core variant, the
    reported baseline) and one core, each repeated for about seconds / 2."""
    import oracle
    out = {}
    for label, th in (("cpu_baseline", 0), ("cpu_baseline_1core", 1)):
        reps, t = 0, 0.0
        while (t < seconds / 2 and reps < 20) or reps == 0:
            t0 = time.perf_counter()
            call(th)
            t += time.perf_counter() - t0
            reps += 1
        out[label] = {"value": work * reps / t, "unit": "effective nnz/s",
                      "cores": oracle.threads() if th == 0 else 1, "kind": "oracle",
                      "sample": f"{what}, {reps} oracle call(s), {t:.1f} s",
                      "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}
    return out


def measure_mttkrp(a, torch, systec, w, name, dev, flush, copy_gbs, with_cpu, steps, warmup):
    """One MTTKRP workload: the prepared call (slot views; the step), its
    kernel, cold times, every algorithm, the one-shot call, the non-symmetric
    kernel on the expanded tensor, errors against the oracle on every element
    and the oracle's own time."""
    order, I = w["order"], w["dim"]
    R = w["B"].shape[1]
    nnz = w["val"].size
    idx = [torch.from_numpy(v).to(dev) for v in w["idx"]]
    val = torch.from_numpy(w["val"].astype(np.float32)).to(dev)
    B32 = torch.from_numpy(w["B"].astype(np.float32)).to(dev)
    B = systec.quantize_bf16(B32) if a.form == "bf16" else B32
    C = torch.empty((I, R), dtype=torch.float32, device=dev)
    hist, eff = systec.expansion_stats(idx, I)
    sb = 2 if a.form == "bf16" else 4
    # compulsory bytes with a pointer over the leading index: pointer + other
    # indices + values + factor read once + output written once
    b_alg = 4 * (I + 1) + nnz * (4 * (order - 1) + 4) + I * R * sb + 4 * I * R
    algo = a.algo
    if algo == "auto":
        algo = systec.mttkrp_choose(I, R, a.form == "bf16", a.path == "prepared")
    t_prep = time.perf_counter()
    T = systec.Tensor.from_coo(idx, val, I)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t_prep
    prepared = lambda: T.mttkrp(B, out=C, algo=algo)  # noqa: E731
    oneshot = lambda: systec.mttkrp(idx, val, B, out=C, algo="atomic")  # noqa: E731
    step, other = (prepared, oneshot) if a.path == "prepared" else (oneshot, prepared)
    kernel_key = f"mttkrp{order}_{algo}" + ("" if a.path == "prepared" else "_oneshot")
    kernel_src = {"views": ("mttkrp.hip", "mttkrp_device.h", "plan.hip"),
                  "atomic": ("mttkrp.hip", "mttkrp_device.h"),
                  "lds": ("mttkrp_lane.hip", "mttkrp_lds.hip", "mttkrp_device.h", "wave_ops.h", "plan.hip")}[algo]
    rec = {"config": {"workload": name, "order": order, "I": I, "R": R, "stored_nnz": nnz,
                      "effective_nnz": eff, "pattern_hist": hist, "B_storage": a.form,
                      "accumulate": "f32", "path": a.path, "algo": algo, "B_alg_bytes": b_alg}}
    _progress(f"{name}: timed region")
    sec = timed(step, steps, warmup)
    rec["value"] = eff / sec
    rec["unit"] = "effective nnz/s"
    rec["ms_per_step"] = sec * 1e3
    rec["config"]["canonical_nnz_per_s"] = nnz / sec
    k_ms, _ = kernel_ms(step, max(10, steps))
    rec["roofline"] = roofline(b_alg, k_ms, kernel_key, kernel_src,
                               f"{kernel_key}:{name}:{a.form}", copy_gbs)
    if a.only_step:
        T.close()
        return rec
    rec["cold"] = cold_ms(torch, step, 20, flush)
    osec = timed(other, max(5, steps // 4), 2)
    rec["other_path"] = {"path": "oneshot" if a.path == "prepared" else "prepared",
                         "ms_per_step": osec * 1e3, "effective_nnz_per_s": eff / osec}
    rec["algos"] = {}
    for alg in ("views", "atomic", "lds"):
        try:
            asec = timed(lambda: T.mttkrp(B, out=C, algo=alg), max(5, steps // 2), 2)  # noqa: E731
            rec["algos"][alg] = {"ms_per_step": asec * 1e3, "effective_nnz_per_s": eff / asec}
        except Exception as e:  # not applicable to this shape
            rec["algos"][alg] = {"error": str(e)}
    if not a.no_compare:
        _progress(f"{name}: non-symmetric comparison")
        try:
            fidx, fval = systec.expand_coo(idx, val, I)
            Cf = torch.empty_like(C)
            csec = timed(lambda: systec.mttkrp_full(fidx, fval, B, out=Cf), steps, warmup)  # noqa: E731
            rec["nonsymmetric"] = {"ms_per_step": csec * 1e3, "effective_nnz_per_s": eff / csec,
                                   "speedup_symmetric": csec / sec,
                                   "expanded_entries": int(fval.numel())}
            del fidx, fval, Cf
            torch.cuda.empty_cache()
        except Exception as e:  # report, do not hide
            rec["nonsymmetric"] = {"error": str(e)}
    import oracle
    step()
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    Bref = B.to(torch.float64).cpu().numpy()
    vref = w["val"].astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    want, _ = oracle.mttkrp(order, I, w["idx"].T, vref, Bref, threads=0)
    t_all = time.perf_counter() - t0
    e2e, _ = oracle.mttkrp(order, I, w["idx"].T, w["val"], w["B"], threads=0)
    rec["oracle_rel_err"] = rel(got, want)
    rec["e2e_rel_err"] = rel(got, e2e)
    if with_cpu:
        # the whole workload on every core; one core on the first k stored
        # entries, about the same time
        legs = cpu_legs(lambda th: oracle.mttkrp(order, I, w["idx"].T, vref, Bref, threads=th),
                        eff, a.cpu_seconds / 2, t_all, "the whole workload")
        rec["cpu_baseline"] = legs["cpu_baseline"]
        k = int(min(nnz, max(1000, nnz * a.cpu_seconds / 4 / max(t_all * oracle.threads(), 1e-3))))
        t0 = time.perf_counter()
        _, cnt = oracle.mttkrp(order, I, w["idx"][:, :k].T, vref[:k], Bref, threads=1)
        t1 = time.perf_counter() - t0
        rec["cpu_baseline_1core"] = {
            "value": cnt["effective_nnz"] / t1, "unit": "effective nnz/s", "cores": 1,
            "kind": "oracle", "sample": f"first {k} of {nnz} stored entries "
                                        f"({cnt['effective_nnz']} expanded), {t1:.1f} s",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}
        # the method's loop over the canonical tuples on one core, same sample
        from oracle import host_loops
        t0 = time.perf_counter()
        host_loops.mttkrp(order, I, w["idx"][:, :k].T, vref[:k], Bref)
        t2 = time.perf_counter() - t0
        v = cnt["effective_nnz"] / t2
        rec["cpu_symmetric_loop_1core"] = {
            "value": v, "unit": "effective nnz/s", "cores": 1, "kind": "host symmetric loop",
            "sample": f"first {k} of {nnz} stored entries, {t2:.2f} s",
            "speedup_vs_expanded_1core": v / rec["cpu_baseline_1core"]["value"]}
    rec["setup_s"] = {"prepare_operand": round(t_prep, 3)}
    T.close()
    return rec


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          f"--gpus {a.gpus} is not supported (sharding across GPUs is not "
                          "part of this benchmark)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    import paper_2406_09266_amd as systec
    from paper_2406_09266_amd import synth

    dev = torch.device("cuda:0")
    if a.workload == "served_mix":
        served_mix(a, torch, systec, synth, dev)
        return
    if a.copy_calibration:
        # a plain device copy of known size, its source pushed out of the
        # last-level cache first, so that FETCH_SIZE/WRITE_SIZE of its
        # dispatch can be compared with the bytes it must move
        src = torch.empty(a.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        fl = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        fl.fill_(0.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, fl
    flush = torch.empty(1 << 27, dtype=torch.float32, device=dev)  # 512 MiB
    copy_gbs = None if a.only_step else copy_ceiling_gbs(torch, dev)
    with_cpu = not a.no_cpu
    t_gen = time.perf_counter()
    w = synth.workload(a.workload)
    t_gen = time.perf_counter() - t_gen
    out = {"metric": "sym sparse MTTKRP/SSYMV effective nnz/s + %HBM peak",
           "unit": "effective nnz/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": a.form, "data": "synthetic (seeded generators; no dataset)"}
    if a.workload.startswith("ssymv"):
        rec = measure_ssymv(a, torch, systec, w, dev, flush, copy_gbs, with_cpu)
    else:
        rec = measure_mttkrp(a, torch, systec, w, a.workload, dev, flush, copy_gbs, with_cpu,
                             a.steps, a.warmup)
    rec.pop("unit", None)
    rec.setdefault("setup_s", {})["generate"] = round(t_gen, 2)
    out.update(rec)
    del w
    # the other workloads, each in its own record of the same line
    subs = [s for s in a.also.split(",") if s and s != a.workload]
    for name in subs:
        _progress(f"{name}: generate")
        t_gen = time.perf_counter()
        ws = synth.workload(name)
        t_gen = time.perf_counter() - t_gen
        r = measure_mttkrp(a, torch, systec, ws, name, dev, flush, copy_gbs, with_cpu,
                           max(10, a.steps), a.warmup)
        r["dtype"] = a.form
        r.setdefault("setup_s", {})["generate"] = round(t_gen, 2)
        out[name] = r
        del ws
    print(json.dumps(out), flush=True)


def served_mix(a, torch, systec, synth, dev):
    """Poisson arrivals of mixed SSYMV / 3-D / 4-D MTTKRP requests against
    resident prepared tensors: the BF16 continuous-batching server versus the
    plain FP32 form (one request at a time, synchronous, FIFO) on the same
    arrival trace. Reports saturation throughput and p50/p99 latency
    (arrival to completion, queueing included) at each offered load."""
    import math
    rng = np.random.Generator(np.random.PCG64(5))
    K = a.pool_per_kind
    t0 = time.perf_counter()
    pool = []  # (kind, operand on device, effective nnz)
    for k in range(K):
        n = int(math.exp(rng.uniform(math.log(1e4), math.log(2e6))))
        deg = rng.uniform(8, 32)
        pool.append(("ssymv", synth.gpu_ssymv_random(n, deg, seed=100 + k, device=dev)))
    for order in (3, 4):
        for k in range(K):
            I = int(math.exp(rng.uniform(math.log(1e3), math.log(2e5))))
            nnz = int(math.exp(rng.uniform(math.log(1e4), math.log(5e7))))
            nnz = min(nnz, int(0.3 * math.comb(I + order - 1, order)))
            pool.append((f"mttkrp{order}",
                         synth.gpu_sym_coo(order, I, nnz, 0.01, seed=200 + 10 * order + k,
                                           device=dev)))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0

    def prepare(item):
        kind, op = item
        if kind == "ssymv":
            return systec.Tensor.from_csr(op["rowptr"], op["col"], op["val"])
        return systec.Tensor.from_coo(op["idx"], op["val"], op["dim"])

    t0 = time.perf_counter()
    served_t = [prepare(it) for it in pool]
    plain_t = [prepare(it) for it in pool]
    t_prep = time.perf_counter() - t0
    eff = [t.effective_nnz for t in served_t]
    dims = [t.dim for t in served_t]
    kinds = [it[0] for it in pool]
    resident = sum(t.bytes for t in served_t)
    # inputs: one per (tensor, R), FP32 and BF16
    Rs = (8, 16, 32)
    inputs = {}
    for p, (kind, op) in enumerate(pool):
        g = torch.Generator(device=dev)
        g.manual_seed(300 + p)
        shapes = [(dims[p],)] if kind == "ssymv" else [(dims[p], R) for R in Rs]
        for shp in shapes:
            x = torch.rand(shp, generator=g, device=dev) * 2 - 1
            inputs[(p, shp[-1] if len(shp) == 2 else 1)] = (x, systec.quantize_bf16(x))
    torch.cuda.synchronize()

    by_kind = {}
    for p, k in enumerate(kinds):
        by_kind.setdefault(k, []).append(p)
    kind_names = sorted(by_kind)

    def draw(count, seed):
        r = np.random.Generator(np.random.PCG64(seed))
        reqs = []
        for _ in range(count):
            k = kind_names[int(r.integers(0, len(kind_names)))]
            p = by_kind[k][int(r.integers(0, len(by_kind[k])))]
            R = 1 if k == "ssymv" else int(r.choice(Rs))
            reqs.append((p, R))
        return reqs

    budget = 200 << 30
    srv = systec.Server(budget_bytes=budget, max_slots=a.max_slots, step_work_nnz=a.step_work,
                        max_inflight=a.max_inflight, streams=a.streams,
                        min_step_work_nnz=a.min_step_work)
    ids = [srv.register(t) for t in served_t]

    def out_for(p, R):
        return torch.empty((dims[p],) if R == 1 else (dims[p], R), device=dev)

    def run_served(reqs, arrivals_s):
        """Submits at the scheduled times; returns the server stats."""
        srv.reset_stats()
        outs = []
        base = systec.Server.now_ns()
        for (p, R), t_arr in zip(reqs, arrivals_s):
            due = base + int(t_arr * 1e9)
            while systec.Server.now_ns() < due:
                pass
            x = inputs[(p, R)][0 if a.served_dtype == "f32" else 1]
            outs.append(srv.submit(ids[p], x, out_for(p, R), arrival_ns=due))
        for rid in outs:
            srv.wait(rid, 600_000_000)
        return srv.stats()

    def run_plain(reqs, arrivals_s):
        lat = []
        base = systec.Server.now_ns()
        last = base
        for (p, R), t_arr in zip(reqs, arrivals_s):
            due = base + int(t_arr * 1e9)
            while systec.Server.now_ns() < due:
                pass
            x = inputs[(p, R)][0]
            t = plain_t[p]
            if kinds[p] == "ssymv":
                t.ssymv(x, out=out_for(p, 1))
            else:
                t.mttkrp(x, out=out_for(p, R))
            torch.cuda.synchronize()
            last = systec.Server.now_ns()
            lat.append((last - due) * 1e-3)
        lat.sort()
        pct = lambda q: lat[max(0, min(len(lat) - 1, math.ceil(q / 100 * len(lat)) - 1))]  # noqa
        span = (last - base) * 1e-9
        eff_done = sum(eff[p] for p, _ in reqs)
        return {"p50_us": pct(50), "p99_us": pct(99), "req_per_s": len(lat) / span,
                "eff_nnz_per_s": eff_done / span}

    def run_plain_async(reqs):
        """The plain kernels back to back with no synchronization between
        requests: the device-bound rate of the one-at-a-time form."""
        outs = [out_for(p, R) for p, R in reqs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (p, R), o in zip(reqs, outs):
            x = inputs[(p, R)][0]
            if kinds[p] == "ssymv":
                plain_t[p].ssymv(x, out=o)
            else:
                plain_t[p].mttkrp(x, out=o)
        torch.cuda.synchronize()
        return len(reqs) / (time.perf_counter() - t0)

    # warm-up, then saturation (everything arrives at once)
    run_served(draw(64, 1), [0.0] * 64)
    n_sat = max(200, a.requests // 3)
    sat_reqs = draw(n_sat, 2)
    st = run_served(sat_reqs, [0.0] * n_sat)
    sat = st["req_per_s"]
    plain_sat = run_plain(sat_reqs, [0.0] * n_sat)
    plain_async = run_plain_async(sat_reqs)
    result = {"metric": "served p50/p99 latency (us) and throughput, BF16 continuous batching "
                        "vs plain FP32 one request at a time",
              "workload": "served_mix", "n_gpus": 1, "data": "synthetic (device generators)",
              "server": {"max_slots": a.max_slots, "step_work_nnz": a.step_work,
                         "max_inflight": a.max_inflight or 2, "streams": a.streams,
                         "min_step_work_nnz": a.min_step_work, "input_dtype": a.served_dtype},
              "pool": {"tensors": len(pool), "per_kind": K, "resident_bytes": resident,
                       "budget_bytes": budget, "effective_nnz_total": int(sum(eff)),
                       "generate_s": round(t_gen, 2), "prepare_s": round(t_prep, 2)},
              "saturation": {"served_req_per_s": sat, "served_eff_nnz_per_s": st["eff_nnz_per_s"],
                             "plain_req_per_s": plain_sat["req_per_s"],
                             "plain_eff_nnz_per_s": plain_sat["eff_nnz_per_s"],
                             "plain_back_to_back_req_per_s": plain_async,
                             "requests": n_sat},
              "loads": []}
    for frac in [float(v) for v in a.loads.split(",") if v]:
        lam = frac * sat
        r = np.random.Generator(np.random.PCG64(int(frac * 1000)))
        arr = np.cumsum(r.exponential(1.0 / lam, a.requests))
        reqs = draw(a.requests, int(frac * 1000) + 7)
        s1 = run_served(reqs, arr)
        p1 = run_plain(reqs, arr)
        result["loads"].append({
            "load": frac, "lambda_req_per_s": lam,
            "served": {"p50_us": s1["p50_us"], "p99_us": s1["p99_us"],
                       "req_per_s": s1["req_per_s"], "eff_nnz_per_s": s1["eff_nnz_per_s"],
                       "steps": s1["steps"], "failed": s1["failed"]},
            "plain": p1})
        print(json.dumps({"progress": f"load {frac} done"}), flush=True)
    srv.close()
    print(json.dumps(result), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
