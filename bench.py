#!/usr/bin/env python3
"""Benchmark of the 3D r2c/c2r path on one MI355X.

One step = one pair: r2c x -> X, then c2r X -> y (with a work buffer, so X is
kept; no feedback from y to x).  The input is a 512^3 real field with a
k^(-5/3) random-phase spectrum (|k| <= 170), unit RMS, seed 3, resident in HBM
before timing starts.  FP32 is the headline line; the FP64 run is reported in
the same line under "f64".

Timing: W untimed warm-up pairs, then K pairs on torch's current stream between
two HIP events, bracketed by device synchronisation.  A second timed region
runs the same K pairs pass by pass (fft3d_run_pass: the same kernels and launch
shapes) with an event pair around every kernel, which gives each kernel's
average duration for the roofline entry.

Roofline: the paper's steps read and write the array once each (plane step:
s*N real + 2*s*M complex; each column pass: 2*s*M in and out), with s the
bytes per real scalar, N = n0*n1*n2 and M = n0*n1*(n2/2+1).  achieved = those
algorithmic bytes of one launch of the dominant kernel / its average duration;
peak = 8 TB/s (MI355X HBM3E).

CPU baseline: the FP64 oracle (oracle/, all host threads) on one pair of the
same field (the sample), reported as pairs/s; the GPU result of that pair is
compared with it (relative L2 over all stored scalars).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "r2c+c2r pairs/s & % HBM peak at 512³ FP32/FP64; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
PASS_NAMES = {0: "plane_r2c", 1: "n1_fwd", 2: "n0_fwd", 3: "n0_inv", 4: "n1_inv", 5: "plane_c2r"}


def pass_bytes(pid: int, shape, elem: int) -> int:
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    M = n0 * n1 * (n2 // 2 + 1)
    if pid in (0, 5):
        return elem * N + 2 * elem * M
    return 4 * elem * M


def pair_bytes_alg(shape, elem: int) -> int:
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    M = n0 * n1 * (n2 // 2 + 1)
    return 2 * (elem * N + 3 * 2 * elem * M)


def pair_bytes_min(shape, elem: int) -> int:
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    M = n0 * n1 * (n2 // 2 + 1)
    return 2 * (elem * N + 2 * elem * M)


# The paper's steps (Sec. 2.1 items 1 and 3, and their inverses) and the
# kernels that make them up; B_alg counts each step as one read and one write
# of the array (steps_alg_bytes), the split plane step spends two sweeps on it.
STEPS = (("a2_plane_r2c", (0, 1)), ("a3_n0_fwd", (2,)), ("a4_n0_inv", (3,)), ("a5_plane_c2r", (4, 5)))


def step_alg_bytes(step: str, shape, elem: int) -> int:
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    M = n0 * n1 * (n2 // 2 + 1)
    if step in ("a2_plane_r2c", "a5_plane_c2r"):
        return elem * N + 2 * elem * M
    return 4 * elem * M


def pair_timer(torch, fn, steps, warmup, s):
    """ms per call of fn on stream s: warm-up, then `steps` calls between two
    events."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_dtype(F, torch, x64, shape, dtype, steps, warmup, fields, coop_plane=False, tuned=False, x_dev=None):
    plan = F.Plan(*shape, dtype=dtype, coop_plane=coop_plane, tuned=tuned)
    desc = plan.describe()
    elem = 4 if dtype == "f32" else 8
    x = x_dev if x_dev is not None else torch.from_numpy(fields.as_dtype(x64, dtype)).to("cuda")
    X = F.empty_complex(plan)
    y = F.empty_real(plan)
    work = F.empty_complex(plan)
    s = torch.cuda.current_stream()

    def pair():
        F.fft3d_r2c(plan, x, X, s)
        F.fft3d_c2r(plan, X, y, work, s)

    for _ in range(warmup):
        pair()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        pair()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps

    # spread: the same number of pairs again, an event after every pair
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    marks[0].record(s)
    for i in range(steps):
        pair()
        marks[i + 1].record(s)
    torch.cuda.synchronize()
    per = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))

    def pct(q):
        return per[min(len(per) - 1, int(round(q * (len(per) - 1))))]

    # per-kernel: the same pairs, pass by pass, an event pair around each kernel
    seq = [(p, x, X) if p == 0 else (p, X, X) for p in desc["r2c_passes"]]
    cur = X
    for p in desc["c2r_passes"]:
        if p == 5:
            seq.append((p, cur, y))
        else:
            seq.append((p, cur, work))
            cur = work
    evs = []
    torch.cuda.synchronize()
    for _ in range(steps):
        for p, a, b in seq:
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record(s)
            F.fft3d_run_pass(plan, p, a, b, s)
            eb.record(s)
            evs.append((p, ea, eb))
    torch.cuda.synchronize()
    tot = {}
    for p, ea, eb in evs:
        tot[p] = tot.get(p, 0.0) + ea.elapsed_time(eb)
    kern = {}
    for p, t in tot.items():
        avg_ms = t / steps
        gbs = pass_bytes(p, shape, elem) / (avg_ms * 1e-3) / 1e9
        # the kernel's own read + write bytes; for the plane and n0 kernels
        # these are the step's algorithmic bytes, the n1 passes are the extra
        # sweep of the split plane step (not in B_alg)
        kern[PASS_NAMES[p]] = {"avg_us": round(avg_ms * 1e3, 2), "swept_bytes": pass_bytes(p, shape, elem),
                               "bytes_are": "swept (extra sweep, not in B_alg)" if p in (1, 4) else "alg",
                               "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # step level: the kernels of each of the paper's steps against its B_alg
    steps_tab = {}
    for name, pids in STEPS:
        us = sum(tot[p] / steps * 1e3 for p in pids if p in tot)
        if us <= 0:
            continue
        ab = step_alg_bytes(name, shape, elem)
        steps_tab[name] = {"kernels": [PASS_NAMES[p] for p in pids if p in tot], "us": round(us, 2),
                           "alg_bytes": ab, "GB_s_alg": round(ab / (us * 1e-6) / 1e9, 1),
                           "frac_alg": round(ab / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    dom = max(tot, key=lambda p: tot[p])
    n = shape[0] * shape[1] * shape[2]
    flops_pair = 2 * 5 * n * math.log2(n)
    b_alg = pair_bytes_alg(shape, elem)
    b_min = pair_bytes_min(shape, elem)
    out = {
        "pairs_s": 1e3 / ms,
        "ms_per_pair": ms,
        "pair_ms_p10_p50_p90": [round(pct(0.1), 4), round(pct(0.5), 4), round(pct(0.9), 4)],
        "hbm_frac_alg": b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "hbm_frac_min": b_min / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "GB_s_alg": b_alg / (ms * 1e-3) / 1e9,
        "gflops": flops_pair / (ms * 1e-3) / 1e9,
        "B_alg_per_pair": b_alg,
        "kernels": kern,
        "steps": steps_tab,
        "dominant": PASS_NAMES[dom],
        "roofline": {"bound": "hbm", "achieved": kern[PASS_NAMES[dom]]["GB_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kern[PASS_NAMES[dom]]["frac"], "traffic": None,
                     "kernel": PASS_NAMES[dom], "alg_bytes_per_launch": pass_bytes(dom, shape, elem),
                     "avg_us": kern[PASS_NAMES[dom]]["avg_us"]},
        "plan": {"plane": desc["plane"]["kind"], "n0_W": desc["n0_pass"]["W"],
                 "coop": desc["plane"].get("coop"), "tuning": desc.get("tuning")},
    }
    # one more pair for the accuracy check against the oracle sample
    pair()
    torch.cuda.synchronize()
    res = (plan, x, X, y)
    return out, res


def run_size(F, torch, shape, dtype, x, steps, warmup, traffic, note):
    """pairs/s of one more (shape, dtype): the tuned plan (the rule unless the
    tuning table has this shape), x resident on the device.  Fractions of the
    HBM peak by B_alg, B_min, the split path's swept bytes and, when a counter
    record of the current sources exists for this configuration, the
    measured bytes."""
    plan = F.Plan(*shape, dtype=dtype, tuned=True)
    X = F.empty_complex(plan)
    y = F.empty_real(plan)
    work = F.empty_complex(plan)
    s = torch.cuda.current_stream()

    def pair():
        F.fft3d_r2c(plan, x, X, s)
        F.fft3d_c2r(plan, X, y, work, s)

    ms = pair_timer(torch, pair, steps, warmup, s)
    elem = 4 if dtype == "f32" else 8
    n = shape[0] * shape[1] * shape[2]
    out = {"shape": list(shape), "dtype": dtype, "note": note, "pairs_s": round(1e3 / ms, 2),
           "ms_per_pair": round(ms, 4), "plane": plan.describe()["plane"]["kind"],
           "gflops": round(2 * 5 * n * math.log2(n) / (ms * 1e-3) / 1e9, 1)}
    for key, b in (("alg", pair_bytes_alg(shape, elem)), ("min", pair_bytes_min(shape, elem)),
                   ("swept", pair_bytes_swept(shape, elem))):
        out["B_" + key] = b
        out["hbm_frac_" + key] = round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    meas = measured_pair_bytes(traffic, shape, dtype)
    out["B_meas"] = meas
    out["hbm_frac_meas"] = round(meas / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if meas else None
    del X, y, work
    return out


def measured_pair_bytes(traffic, shape, dtype):
    """Counter bytes (fetch + write, calibrated) of one pair's kernels, from
    the committed counter record of the current sources, or None."""
    rec = ((traffic or {}).get("configs") or {}).get("x".join(map(str, shape)), {}).get(dtype)
    if not rec:
        return None
    return int(sum(k["fetch_bytes"] + k["write_bytes"] for k in rec.values()))


def run_ablation(F, torch, x64, shape, dtype, steps, warmup, fields, free_ms):
    """The paper's comparison (Sec. 3) on one GPU: the transpose-based method
    (Sec. 2.1: plane step, explicit n0<->n1 exchange, n0 columns of the
    exchanged layout; inverse in reverse) against the transpose-free path
    (Sec. 2.2) timed above, same kernels otherwise, same field."""
    plan = F.Plan(*shape, dtype=dtype)
    n0, n1, n2 = shape
    x = torch.from_numpy(fields.as_dtype(x64, dtype)).to("cuda")
    Xt = torch.empty((n1, n0, n2 // 2 + 1), dtype=F.torch_dtypes(dtype)[1], device="cuda")
    y = F.empty_real(plan)
    work = F.empty_complex(plan)
    s = torch.cuda.current_stream()

    def pair():
        F.fft3d_r2c_transposed(plan, x, Xt, work, s)
        F.fft3d_c2r_transposed(plan, Xt, y, work, s)

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(k):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms = timed(pair, steps)
    swap_us = 1e3 * timed(lambda: F.fft3d_run_pass(plan, F.FFT3D_PASS_SWAP01, work, Xt, s), steps)
    n0t_us = 1e3 * timed(lambda: F.fft3d_run_pass(plan, F.FFT3D_PASS_N0T_FWD, Xt, Xt, s), steps)
    elem = 4 if dtype == "f32" else 8
    M = n0 * n1 * (n2 // 2 + 1)
    del x, Xt, y, work
    return {"transpose_based_ms_per_pair": round(ms, 4), "transpose_free_ms_per_pair": round(free_ms, 4),
            "transpose_free_speedup": round(ms / free_ms, 3),
            "exchange_us": round(swap_us, 1), "exchange_GB_s": round(4 * elem * M / (swap_us * 1e-6) / 1e9, 1),
            "n0_columns_exchanged_layout_us": round(n0t_us, 1)}


def _box_counts(shape, kmax):
    n0, n1, n2 = shape
    K0, K1, K2 = kmax
    hw = n2 // 2 + 1 if K2 < 0 or K2 >= n2 // 2 else K2 + 1
    m1 = n1 if K1 < 0 or 2 * K1 + 1 >= n1 else 2 * K1 + 1
    m0 = n0 if K0 < 0 or 2 * K0 + 1 >= n0 else 2 * K0 + 1
    return hw, m1, m0


def pruned_pair_bytes_alg(shape, elem: int, kmax) -> int:
    """B_alg of a pruned pair, in the same accounting as pair_bytes_alg (each
    of the paper's two steps reads and writes once): step 1 reads the real
    array and writes the kept (k1, k2) of every plane, step 3 reads those and
    writes the kept box; the inverse mirrors it."""
    n0, n1, n2 = shape
    hw, m1, m0 = _box_counts(shape, kmax)
    c = 2 * elem
    return 2 * (elem * n0 * n1 * n2 + c * (2 * n0 * m1 * hw + m0 * m1 * hw))


def pruned_pair_bytes_swept(shape, elem: int, kmax) -> int:
    """Bytes a pruned pair moves on the split plane path (rows kernel, n1
    pass, n0 pass, each reading and writing only inside the box)."""
    n0, n1, n2 = shape
    hw, m1, m0 = _box_counts(shape, kmax)
    c = 2 * elem
    return 2 * (elem * n0 * n1 * n2 + c * (2 * n0 * n1 * hw + 2 * n0 * m1 * hw + m0 * m1 * hw))


def pair_bytes_swept(shape, elem: int) -> int:
    """Bytes a full pair moves on the split plane path (three sweeps)."""
    n0, n1, n2 = shape
    M = n0 * n1 * (n2 // 2 + 1)
    return 2 * (elem * n0 * n1 * n2 + 5 * 2 * elem * M)


def run_pruned(F, torch, x64, shape, dtype, steps, warmup, fields, free_ms):
    """Pruned pair (forward writes, inverse reads, only the two-thirds box
    |k| <= n/3) against the full pair timed above, same field."""
    plan = F.Plan(*shape, dtype=dtype)
    kmax = tuple(n // 3 for n in shape)
    x = torch.from_numpy(fields.as_dtype(x64, dtype)).to("cuda")
    X = F.empty_complex(plan)
    y = F.empty_real(plan)
    work = F.empty_complex(plan)
    s = torch.cuda.current_stream()

    def pair():
        F.fft3d_r2c_pruned(plan, x, X, kmax, s)
        F.fft3d_c2r_pruned(plan, X, y, kmax, work, s)

    for _ in range(warmup):
        pair()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        pair()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    elem = 4 if dtype == "f32" else 8
    b = pruned_pair_bytes_alg(shape, elem, kmax)
    bs = pruned_pair_bytes_swept(shape, elem, kmax)
    del x, X, y, work
    return {"kmax": list(kmax), "ms_per_pair": round(ms, 4), "pairs_s": round(1e3 / ms, 2),
            "full_ms_per_pair": round(free_ms, 4), "speedup_vs_full": round(free_ms / ms, 3),
            "bytes_alg": b, "bytes_ratio_vs_full": round(b / pair_bytes_alg(shape, elem), 3),
            "bytes_swept": bs, "swept_ratio_vs_full": round(bs / pair_bytes_swept(shape, elem), 3),
            "GB_s_alg": round(b / (ms * 1e-3) / 1e9, 1), "GB_s_swept": round(bs / (ms * 1e-3) / 1e9, 1)}


def batch_items(F, torch, fields, count=64, seed=4):
    """The mixed batch's items: `count` fields drawn from fields.batch_mix,
    uniform[-1,1] values (field i: seed 1000+i), each a ROUNDTRIP item (r2c
    then c2r with work).  Returns (mix, plans, items, B_alg, real points)."""
    mix = fields.batch_mix(count, seed)
    plans, items = {}, []
    b_alg = 0
    points = 0
    for i, (shape, dt) in enumerate(mix):
        if (shape, dt) not in plans:
            plans[(shape, dt)] = F.Plan(*shape, dtype=dt)
        p = plans[(shape, dt)]
        x = torch.from_numpy(fields.as_dtype(fields.uniform(shape, 1000 + i), dt)).to("cuda")
        items.append((p, F.FFT3D_ROUNDTRIP, x, F.empty_complex(p), F.empty_real(p), F.empty_complex(p)))
        b_alg += pair_bytes_alg(shape, 4 if dt == "f32" else 8)
        points += shape[0] * shape[1] * shape[2]
    return mix, plans, items, b_alg, points


def batch_traffic_run(F, torch, fields, launches):
    """For the batch's counter profile (profiles/fft3d_batch_traffic.md): a
    1 GiB device copy (the counters' calibration), then `launches` launches
    of the 64-field batch handle; one JSON line."""
    mix, plans, items, b_alg, points = batch_items(F, torch, fields)
    handle = F.Batch(items)
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    for _ in range(launches):
        handle.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    print(json.dumps({"batch_launches": launches, "B_alg": b_alg, "launches": len(handle.describe()["launches"]),
                      "status": handle.status()}), flush=True)
    return 0


def run_batch(F, torch, fields, steps, warmup, count=64, seed=4):
    """The mixed batch: `count` fields drawn from fields.batch_mix (shapes
    32^3 .. 192x192x96, FP32/FP64), uniform[-1,1] values (field i: seed
    1000+i), each a ROUNDTRIP item (r2c then c2r with work).  Times the
    batched launch of the whole batch (the rule's level mode: graph replay of
    a batch handle, and the ring-staged fft3d_batch_submit) against the same items launched field
    by field (the items' own kernels, FFT3D_BATCH_SEQUENTIAL), and the launch
    shape the batch autotuner picks.  Returns (one item per (shape, dtype)
    with the outputs of the last launch, the record)."""
    mix, plans, items, b_alg, points = batch_items(F, torch, fields, count, seed)
    s = torch.cuda.current_stream()
    handle = F.Batch(items)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def ring_submit():
        # the submit never waits: with every ring slot in flight it returns
        # FFT3D_ERR_BUSY, and the caller tries again
        while True:
            try:
                return F.fft3d_batch_submit(items, s)
            except F.Fft3dError as e:
                if e.code != F.FFT3D_ERR_BUSY:
                    raise
                time.sleep(1e-4)

    ms_graph = timed(lambda: handle.launch(s))
    ms_ring = timed(ring_submit)
    ms_seq = timed(lambda: F.fft3d_batch_submit_ex(items, F.FFT3D_BATCH_SEQUENTIAL, s))
    status = handle.status()
    desc = handle.describe()
    # the batch autotuner's launch shape, as a graph-launched handle
    bt, rep = F.fft3d_batch_autotune(items, effort=0)
    tuned_handle = F.Batch(items, tuning=bt)
    ms_tuned = timed(lambda: tuned_handle.launch(s))
    status_tuned = tuned_handle.status()
    # the outputs of the last launch: FP32 items against the plain FP64 path
    # on the same GPU (the FP32 input upcast), one item per shape
    fp64_cmp, seen = {}, set()
    for i, (shape, dt) in enumerate(mix):
        if dt != "f32" or shape in seen:
            continue
        seen.add(shape)
        p, _, x, mid, out, w = items[i]
        p64 = F.Plan(*shape, dtype="f64")
        X64 = F.r2c(p64, x.double())
        y64 = F.c2r(p64, X64.clone(), work=F.empty_complex(p64))
        torch.cuda.synchronize()
        fp64_cmp["x".join(map(str, shape))] = {
            "rel_l2_r2c": float(torch.linalg.vector_norm((mid.to(torch.complex128) - X64).ravel()) /
                                torch.linalg.vector_norm(X64.ravel())),
            "rel_l2_c2r": float(torch.linalg.vector_norm((out.double() - y64).ravel()) /
                                torch.linalg.vector_norm(y64.ravel()))}
    gbs = b_alg / (ms_graph * 1e-3) / 1e9
    samples = []
    seen = set()
    for i, (shape, dt) in enumerate(mix):
        if (shape, dt) not in seen:
            seen.add((shape, dt))
            samples.append((shape, dt, items[i]))
    rec = {
        "workload": "%d fields (seed %d) of %s, FP32/FP64 mixed (%d FP64), %.1f M real points, ROUNDTRIP "
                    "items" % (count, seed, "/".join("x".join(map(str, sh)) for sh in fields.BATCH_SHAPES),
                               sum(d == "f64" for _, d in mix), points / 1e6),
        "fields_s": round(count * 1e3 / ms_graph, 1),
        "ms_per_launch": round(ms_graph, 4),
        "ms_ring_submit": round(ms_ring, 4),
        "ms_per_field_launches": round(ms_seq, 4),
        "speedup_vs_per_field": round(ms_seq / ms_graph, 3),
        "B_alg": b_alg,
        "GB_s_alg": round(gbs, 1),
        "hbm_frac_alg": round(gbs / HBM_PEAK_GBS, 4),
        "grid": desc["grid"], "tickets": desc["tickets"], "tasks": len(desc["tasks"]), "lds": desc["lds"],
        "launches": len(desc.get("launches", [])), "mode": desc["mode"],
        "status": status,
        "tuned": {"batch_tuning": bt, "ms_per_launch": round(ms_tuned, 4), "fields_s": round(count * 1e3 / ms_tuned, 1),
                  "GB_s_alg": round(b_alg / (ms_tuned * 1e-3) / 1e9, 1), "speedup_vs_rule": round(ms_graph / ms_tuned, 3),
                  "status": status_tuned, "candidates": len(rep["candidates"])},
        "f32_vs_plain_f64_gpu": fp64_cmp,
    }
    # counter bytes per launch, from the committed record of the same sources
    tr = recorded_batch_traffic()
    if tr and tr.get("B_alg") == b_alg:
        rec["B_meas_per_launch"] = tr["bytes_per_launch"]
        rec["meas_over_alg"] = round(tr["bytes_per_launch"] / b_alg, 4)
        rec["hbm_frac_meas"] = round(tr["bytes_per_launch"] / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    else:
        rec["B_meas_per_launch"] = None
    # samples: one item per (shape, dtype) with the outputs of the last
    # launch, for the oracle leg
    return samples, rec


def served_bytes_alg(shape, dtype, direction, ncomp=3) -> int:
    """Algorithmic bytes of one request: the passes of one direction (half a
    pair), per field."""
    return ncomp * pair_bytes_alg(shape, 4 if dtype == "f32" else 8) // 2


def run_served(F, torch, fields, rate=200.0, measured=2000, warmup_s=5.0, seed=5, budget=200 * 10**9,
               nstreams=4, log=None):
    """The served stream: Poisson arrivals of mean `rate`/s of 3-component
    velocity-field requests (fields.serve_mix: shapes 64^3 .. 512^3, 2% 1024^3
    FP32, 80/20 FP32/FP64, r2c or c2r), admitted under an HBM budget, run by
    the library's server (continuous batching on `nstreams` streams).  Inputs
    are resident pools, one 3-component field and one 3-component spectrum
    per (shape, dtype) (fields.velocity_pool_torch).  The first warmup_s
    seconds of arrivals are not measured; then `measured` requests.
    Latency = done - arrival (server clock)."""
    import threading
    import numpy as np

    n_warm = int(rate * warmup_s)
    count = n_warm + measured
    arrive, reqs = fields.serve_mix(count, rate, seed)
    keys = sorted({(s, d) for s, d, _ in reqs})
    pools = {}
    t0 = time.time()
    for i, (s, d) in enumerate(keys):
        u, U = fields.velocity_pool_torch(s, 2000 + i, d)
        pools[(s, d)] = ([u[c] for c in range(3)], [U[c] for c in range(3)])
        torch.cuda.synchronize()
    if log:
        log("# served pools: %d (shape, dtype) in %.1f s" % (len(keys), time.time() - t0))
    torch.cuda.empty_cache()
    srv = None
    while srv is None:
        try:
            srv = F.Server(budget, nstreams=nstreams)
        except F.Fft3dError:
            if budget <= 16 * 10**9:
                raise
            budget = budget * 3 // 4  # what the device has left after the pools
    if log:
        log("# served budget %.1f GB" % (budget / 1e9))
    # plans and first launches outside the measurement
    for s, d in keys:
        for r in (0, 1):
            rid = srv.submit(s, d, r, pools[(s, d)][r])
            srv.wait(rid, 120.0)
            srv.release(rid)
    ids = [None] * count
    done = [None] * count
    errors = []

    def producer():
        start = time.perf_counter()
        for i in range(count):
            dt = start + arrive[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            s, d, r = reqs[i]
            ids[i] = srv.submit(s, d, r, pools[(s, d)][r])

    def consumer():
        try:
            for i in range(count):
                while ids[i] is None:
                    time.sleep(5e-5)
                srv.wait(ids[i], 300.0)
                _, t = srv.result(ids[i], 3)
                done[i] = t
                srv.release(ids[i])
        except Exception as e:
            errors.append(e)

    tp = threading.Thread(target=producer)
    tc = threading.Thread(target=consumer)
    tp.start()
    tc.start()
    tp.join()
    tc.join()
    st = srv.stats()
    srv.close()
    if errors:
        raise errors[0]
    meas = list(range(n_warm, count))
    lat = np.array([done[i][3] - done[i][0] for i in meas])
    qwait = np.array([done[i][1] - done[i][0] for i in meas])
    # completions per second while the measured requests complete (under
    # overload the backlog ahead of them is not counted against the GPU)
    t_done = sorted(done[i][3] for i in meas)
    span = max(t_done[-1] - t_done[0], 1e-9) * len(meas) / max(len(meas) - 1, 1)
    nbytes = sum(served_bytes_alg(*reqs[i]) for i in meas)
    del pools
    torch.cuda.empty_cache()
    return {
        "workload": "Poisson arrivals at %.0f/s of 3-component k^-5/3 velocity-field requests: shapes %s, "
                    "plus %s FP32 with probability 0.02; 80/20 FP32/FP64; r2c or c2r 50/50; budget %.0f GB; "
                    "%d warm-up + %d measured requests (seed %d)" % (
                        rate, "/".join("x".join(map(str, s)) for s in fields.SERVE_SHAPES),
                        "x".join(map(str, fields.SERVE_LARGE)), budget / 1e9, n_warm, measured, seed),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "mean_ms": round(float(lat.mean()) * 1e3, 3),
        "p99_queue_ms": round(float(np.percentile(qwait, 99)) * 1e3, 3),
        "offered_req_s": round(rate, 1),
        "completed_req_s": round(len(meas) / span, 1),
        "GB_s_alg": round(nbytes / span / 1e9, 1),
        "peak_reserved_GB": round(st["peak_reserved_bytes"] / 1e9, 3),
        "budget_GB": round(st["budget_bytes"] / 1e9, 3),
        "batched_launches": st["batched_launches"],
        "single_launches": st["single_launches"],
    }


def served_samples(F, torch, fields, budget=16 * 10**9):
    """A few requests through a server (both directions, both dtypes, shapes
    up to 128^3) with inputs from the numpy generators, so that the oracle
    leg can check them; FP32 ones are also compared with the plain FP64 path
    on the same GPU.  Returns (records, host data for the oracle leg)."""
    import numpy as np
    cases = [((64, 64, 64), "f32"), ((64, 64, 64), "f64"), ((128, 128, 128), "f32"), ((96, 96, 96), "f64")]
    srv = F.Server(budget, nstreams=2)
    recs, host = [], []
    try:
        for k, (shape, dt) in enumerate(cases):
            for direction in (0, 1):
                seed = 2500 + 2 * k + direction
                if direction == 0:
                    inp = fields.as_dtype(fields.velocity_field(shape, seed), dt)
                else:
                    inp = fields.as_dtype(fields.velocity_spectrum(shape, seed), dt)
                dev = [torch.from_numpy(np.ascontiguousarray(inp[c])).to("cuda") for c in range(3)]
                rid = srv.submit(shape, dt, direction, dev)
                srv.wait(rid, 120.0)
                addrs, _ = srv.result(rid, 3)
                rdt, cdt = F.torch_dtypes(dt)
                n0, n1, n2 = shape
                oshape, odt = ((n0, n1, n2 // 2 + 1), cdt) if direction == 0 else ((n0, n1, n2), rdt)
                outs = []
                for c in range(3):
                    t = torch.empty(oshape, dtype=odt, device="cuda")
                    F.copy_from_device(t, addrs[c], t.numel() * t.element_size())
                    outs.append(t.cpu().numpy())
                srv.release(rid)
                rec = {"shape": list(shape), "dtype": dt, "dir": "r2c" if direction == 0 else "c2r"}
                if dt == "f32":
                    p64 = F.Plan(*shape, dtype="f64")
                    errs = []
                    for c in range(3):
                        a = dev[c].to(torch.complex128 if direction else torch.float64)
                        ref = F.r2c(p64, a) if direction == 0 else F.c2r(p64, a.clone(), work=F.empty_complex(p64))
                        torch.cuda.synchronize()
                        r = ref.cpu().numpy()
                        errs.append(float(np.linalg.norm((outs[c].astype(r.dtype) - r).ravel()) / np.linalg.norm(r.ravel())))
                    rec["rel_l2_vs_plain_f64_gpu"] = max(errs)
                recs.append(rec)
                host.append((shape, dt, direction, inp, outs))
    finally:
        srv.close()
    return recs, host


# The configurations whose counter bytes profiles/fft3d_pair_traffic.md records.
TRAFFIC_CONFIGS = (((512, 512, 512), "f32"), ((512, 512, 512), "f64"), ((256, 256, 256), "f64"),
                   ((1024, 1024, 1024), "f32"), ((1024, 1024, 1024), "f64"))
# The sources of the pair's kernels: the two translation units that build
# them and every header they include.
DEVICE_SOURCES = ("fft3d_kern_f32.hip", "fft3d_kern_f64.hip", "fft3d_kernels.hpp", "fft3d_device.hpp",
                  "fft3d_sched.hpp", "fft3d_internal.hpp")


def _code_only(text: str) -> bytes:
    """Source text without comments and with whitespace collapsed: what the
    compiler sees (a comment edit leaves the identity unchanged)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split()).encode()


def kernel_source_sha256() -> str:
    """Identity of what the counters measured: the device code of the pair's
    kernels (their .hip files and the headers they include, comments
    stripped) and the launch shapes of the rule plans of the recorded
    configurations (their descriptions).  A counter record taken on another
    identity is stale."""
    import hashlib
    from paper_1406_5597_amd import fft3d as F
    d = os.path.join(ROOT, "paper_1406_5597_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(DEVICE_SOURCES):
        h.update(name.encode())
        h.update(_code_only(open(os.path.join(d, name)).read()))
    h.update(_code_only(open(os.path.join(ROOT, "include", "fft3d.h")).read()))
    for shape, dt in TRAFFIC_CONFIGS:
        desc = F.Plan(*shape, dtype=dt, host_only=True).describe()
        desc.pop("device", None)
        h.update(json.dumps(desc, sort_keys=True).encode())
    return h.hexdigest()


# The sources of the level mode's launches and of the batch's tiling: what
# the batch's counter record (profiles/fft3d_batch_traffic.md) depends on.
BATCH_SOURCES = ("fft3d_level.hip", "fft3d_batch_tiles.hpp", "fft3d_batch.hpp", "fft3d_kernels.hpp",
                 "fft3d_device.hpp", "fft3d_sched.hpp", "fft3d_internal.hpp", "fft3d_batch_host.cpp",
                 "fft3d_batch_host.hpp", "fft3d_plan.cpp")


def batch_source_sha256() -> str:
    """Identity of the batch's counter record: the level mode's device code,
    the host code that tiles and schedules the batch (comments stripped)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1406_5597_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(BATCH_SOURCES):
        h.update(name.encode())
        h.update(_code_only(open(os.path.join(d, name)).read()))
    h.update(_code_only(open(os.path.join(ROOT, "include", "fft3d.h")).read()))
    return h.hexdigest()


def recorded_batch_traffic():
    """The batch's HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by
    the copy calibration) from the committed rocprofv3 summary, if it was
    taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", "fft3d_batch_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            return rec if rec.get("source_sha256") == batch_source_sha256() else None
    return None


def recorded_traffic():
    """Per-kernel HBM bytes (FETCH_SIZE and WRITE_SIZE, scaled by the copy
    calibration) from the committed rocprofv3 summary, if it was taken on the
    current sources; else None."""
    path = os.path.join(ROOT, "profiles", "fft3d_pair_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            return rec if rec.get("source_sha256") == kernel_source_sha256() else None
    return None


def copy_bandwidth(torch) -> float:
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-batch measurement")
    ap.add_argument("--no-ablation", action="store_true", help="skip the transpose-based comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream measurement")
    ap.add_argument("--no-pruned", action="store_true", help="skip the pruned (two-thirds box) pair")
    ap.add_argument("--serve-rates", default="200", help="comma-separated arrival rates (req/s) of the served stream")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per served rate")
    ap.add_argument("--serve-warmup", type=float, default=10.0, help="seconds of unmeasured arrivals first")
    ap.add_argument("--no-tune", action="store_true", help="time the rule plans only (no autotuner run)")
    ap.add_argument("--no-sizes", action="store_true", help="skip the 256^3 FP64 and 1024^3 lines")
    ap.add_argument("--coop-plane", action="store_true",
                    help="cooperative one-launch plane step for large planes instead of the two kernels")
    ap.add_argument("--batch-traffic", type=int, default=0, metavar="K",
                    help="only the batch's counter-profile run: a 1 GiB copy, then K launches of the 64-field "
                         "batch handle (no metric line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU form (the slab exchange "
              "across devices is a design, not built); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1406_5597_amd import fft3d as F
    from workloads import fields

    F.fft3d_init()  # the device's batch ring
    if args.batch_traffic > 0:
        return batch_traffic_run(F, torch, fields, args.batch_traffic)
    n = args.size
    shape = (n, n, n)
    t0 = time.time()
    x64 = fields.k53_field(shape, seed=3)
    print("# field %s generated in %.1f s" % (shape, time.time() - t0), file=sys.stderr, flush=True)
    dtypes = [d for d in args.dtypes.split(",") if d]
    traffic = recorded_traffic()
    results, keep, tune = {}, {}, {}
    for d in dtypes:
        tuned = not args.coop_plane and not args.no_tune
        if tuned:
            # the autotuner first (its winner enters the tuning table; the
            # rule is kept unless a candidate is faster)
            t0 = time.time()
            best, rep = F.autotune(shape, d, effort=0)
            tune[d] = {"tuning": best, "kept": rep["kept"], "search_s": round(time.time() - t0, 2),
                       "candidates": len(rep["candidates"]), "pair_ms_rule": rep["pair_ms_rule"],
                       "pair_ms_tuned": rep["pair_ms_tuned"]}
            print("# autotune %s: kept %s (%s), %.1f s" % (d, rep["kept"], best, time.time() - t0),
                  file=sys.stderr, flush=True)
        print("# timing %s ..." % d, file=sys.stderr, flush=True)
        results[d], keep[d] = run_dtype(F, torch, x64, shape, d, args.steps, args.warmup, fields,
                                        args.coop_plane, tuned=tuned)
        if tuned:
            # the rule plan on the same input, for comparison
            rp = F.Plan(*shape, dtype=d)
            plan_t, xt, Xt_, yt = keep[d]
            wt = F.empty_complex(rp)
            st = torch.cuda.current_stream()
            ms_rule = pair_timer(torch, lambda: (F.fft3d_r2c(rp, xt, Xt_, st), F.fft3d_c2r(rp, Xt_, yt, wt, st)),
                                 args.steps, args.warmup, st)
            # leave the tuned plan's last pair in X and y for the accuracy check
            F.fft3d_r2c(plan_t, xt, Xt_, st)
            F.fft3d_c2r(plan_t, Xt_, yt, wt, st)
            torch.cuda.synchronize()
            del wt, rp
            tune[d]["bench_ms_rule"] = round(ms_rule, 4)
            tune[d]["bench_ms_tuned"] = round(results[d]["ms_per_pair"], 4)
            tune[d]["speedup_vs_rule"] = round(ms_rule / results[d]["ms_per_pair"], 4)
        print("# %s: %.3f ms/pair, %.1f pairs/s, dominant %s %.1f GB/s" % (
            d, results[d]["ms_per_pair"], results[d]["pairs_s"], results[d]["dominant"],
            results[d]["roofline"]["achieved"]), file=sys.stderr, flush=True)
    sizes = None
    if not args.no_sizes:
        sizes = []
        # 256^3 FP64 (k^-5/3 field, |k| <= 85, seed 2): its working set is
        # about the size of the 256 MB memory-side cache (cache-assisted)
        s3 = (256, 256, 256)
        x256 = torch.from_numpy(fields.k53_field(s3, seed=2, kmax=85)).to("cuda")
        if not args.no_tune:
            F.autotune(s3, "f64", effort=0)
        sizes.append(run_size(F, torch, s3, "f64", x256, args.steps, args.warmup, traffic,
                              "k^-5/3 field |k|<=85 seed 2; working set ~ the 256 MB memory-side cache: "
                              "cache-assisted"))
        del x256
        # 1024^3: a uniform[-1,1] field made on the device (torch generator,
        # seed 3); the pair's time does not depend on the values (the parity
        # tests compare the 1024^3 k^-5/3 outputs with the oracle)
        s4 = (1024, 1024, 1024)
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        for d in dtypes:
            rdt = torch.float32 if d == "f32" else torch.float64
            xb = torch.rand(s4, generator=g, device="cuda", dtype=rdt) * 2 - 1
            if not args.no_tune:
                F.autotune(s4, d, effort=0)
            sizes.append(run_size(F, torch, s4, d, xb, max(5, args.steps // 5), min(args.warmup, 3), traffic,
                                  "uniform[-1,1] made on the device (torch seed 3)"))
            del xb
            torch.cuda.empty_cache()
        for z in sizes:
            print("# size %s %s: %.2f pairs/s (%.1f%% of peak by B_alg)" % (
                z["shape"], z["dtype"], z["pairs_s"], 100 * z["hbm_frac_alg"]), file=sys.stderr, flush=True)
    ablation = None
    if not args.no_ablation:
        ablation = {}
        for d in dtypes:
            print("# transpose-based method %s ..." % d, file=sys.stderr, flush=True)
            ablation[d] = run_ablation(F, torch, x64, shape, d, args.steps, args.warmup, fields,
                                       results[d]["ms_per_pair"])
            print("# %s: transpose-based %.3f ms/pair vs transpose-free %.3f" % (
                d, ablation[d]["transpose_based_ms_per_pair"], results[d]["ms_per_pair"]), file=sys.stderr,
                flush=True)
    pruned = None
    if not args.no_pruned:
        pruned = {}
        for d in dtypes:
            print("# pruned pair %s ..." % d, file=sys.stderr, flush=True)
            pruned[d] = run_pruned(F, torch, x64, shape, d, args.steps, args.warmup, fields,
                                   results[d]["ms_per_pair"])
            print("# %s: pruned %.3f ms/pair vs full %.3f (%.2fx), %.1f GB/s alg" % (
                d, pruned[d]["ms_per_pair"], results[d]["ms_per_pair"], pruned[d]["speedup_vs_full"],
                pruned[d]["GB_s_alg"]), file=sys.stderr, flush=True)
    copy_gbs = copy_bandwidth(torch)
    batch = None
    if not args.no_batch:
        print("# mixed batch ...", file=sys.stderr, flush=True)
        batch_samples, batch = run_batch(F, torch, fields, args.steps, args.warmup)
        print("# batch: %.3f ms/launch (%.1f fields/s, %.1f GB/s), per-field launches %.3f ms" % (
            batch["ms_per_launch"], batch["fields_s"], batch["GB_s_alg"], batch["ms_per_field_launches"]),
            file=sys.stderr, flush=True)

    served = None
    served_acc, served_host = None, None
    if not args.no_serve:
        print("# served samples ...", file=sys.stderr, flush=True)
        served_acc, served_host = served_samples(F, torch, fields)
        served = []
        for rate in [float(v) for v in args.serve_rates.split(",") if v]:
            print("# served stream at %.0f req/s ..." % rate, file=sys.stderr, flush=True)
            sv = run_served(F, torch, fields, rate=rate, measured=args.serve_requests, warmup_s=args.serve_warmup,
                            log=lambda m: print(m, file=sys.stderr, flush=True))
            print("# served: p50 %.3f ms, p99 %.3f ms, %.1f req/s" % (sv["p50_ms"], sv["p99_ms"],
                                                                       sv["completed_req_s"]),
                  file=sys.stderr, flush=True)
            served.append(sv)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        head = dtypes[0]
        plan, x, X, y = keep[head]
        xin = fields.as_dtype(x64, head).astype(np.float64)
        print("# oracle sample (%s pairs, FP64, about 10 s) ..." % (shape,), file=sys.stderr, flush=True)
        t0 = time.time()
        pairs = 0
        while True:
            Xo = oracle.r2c(xin)
            yo = oracle.c2r(Xo, n)
            pairs += 1
            if time.time() - t0 >= 10.0 or pairs >= 8:
                break
        dt = time.time() - t0
        cpu = {"value": pairs / dt, "unit": "pairs/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": "%d r2c+c2r pairs of the same %dx%dx%d field (%s-rounded input, computed in FP64), "
                         "%.1f s wall" % (pairs, n, n, n, head, dt)}
        for d in dtypes:
            p, xd, Xd, yd = keep[d]
            if d != head:
                continue
            results[d]["rel_l2_r2c"] = fields.rel_l2(Xd.cpu().numpy(), Xo)
            results[d]["rel_l2_c2r"] = fields.rel_l2(yd.cpu().numpy(), yo)
        del Xo, yo
        # every other dtype: one oracle pair on its own input
        for d in dtypes:
            if d == head:
                continue
            p, xd, Xd, yd = keep[d]
            xin_d = fields.as_dtype(x64, d).astype(np.float64)
            Xo = oracle.r2c(xin_d)
            yo = oracle.c2r(Xo, n)
            results[d]["rel_l2_r2c"] = fields.rel_l2(Xd.cpu().numpy(), Xo)
            results[d]["rel_l2_c2r"] = fields.rel_l2(yd.cpu().numpy(), yo)
            del Xo, yo
        # the batch: one item per (shape, dtype), outputs of the last launch
        if batch is not None:
            acc = {}
            for shp, dt_, it in batch_samples:
                p, _, xb, mid, out, w = it
                xin_b = xb.cpu().numpy().astype(np.float64)
                Xo = oracle.r2c(xin_b)
                yo = oracle.c2r(Xo, shp[2])
                acc["%s_%s" % ("x".join(map(str, shp)), dt_)] = {
                    "rel_l2_r2c": fields.rel_l2(mid.cpu().numpy(), Xo), "rel_l2_c2r": fields.rel_l2(out.cpu().numpy(), yo)}
            batch["rel_l2_vs_oracle"] = acc
        # served samples: every component of each request
        if served_host is not None:
            for rec, (shp, dt_, direction, inp, outs) in zip(served_acc, served_host):
                errs = []
                for c in range(3):
                    a = inp[c].astype(np.complex128 if direction else np.float64)
                    ref = oracle.r2c(a) if direction == 0 else oracle.c2r(a, shp[2])
                    errs.append(fields.rel_l2(outs[c], ref))
                rec["rel_l2_vs_oracle"] = max(errs)
        # smaller configurations, one thread and all threads (seconds per pair)
        small = {}
        for m in (32, 256):
            xs = fields.uniform((m, m, m), 1)
            row = {}
            for th in (1, 0):
                t1 = time.time()
                oracle.c2r(oracle.r2c(xs, th), m, th)
                row["threads_%d" % (th or oracle.max_threads())] = round(time.time() - t1, 4)
            small["%d^3" % m] = row
        # the benchmark size on one thread (one pair), beside the all-thread rate above
        t1 = time.time()
        oracle.c2r(oracle.r2c(xin, 1), n, 1)
        small["%d^3" % n] = {"threads_1": round(time.time() - t1, 3), "threads_%d" % oracle.max_threads():
                             round(1.0 / cpu["value"], 3)}
        cpu["pair_seconds_fp64"] = small

    for d in dtypes:
        roof = results[d]["roofline"]
        rec = ((traffic or {}).get("configs") or {}).get("x".join(map(str, shape)), {}).get(d, {})
        t = rec.get(roof["kernel"])
        if t:
            roof["traffic"] = int(t["fetch_bytes"] + t["write_bytes"])
            roof["traffic_fetch"] = int(t["fetch_bytes"])
            roof["traffic_write"] = int(t["write_bytes"])
        meas = measured_pair_bytes(traffic, shape, d)
        elem = 4 if d == "f32" else 8
        ms = results[d]["ms_per_pair"]
        results[d]["hbm_frac_swept"] = pair_bytes_swept(shape, elem) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        results[d]["B_meas_per_pair"] = meas
        results[d]["hbm_frac_meas"] = meas / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS if meas else None
    head = dtypes[0]
    r = results[head]
    line = {
        "metric": METRIC,
        "value": round(r["pairs_s"], 2),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_pair"], 4),
        "pair_ms_p10_p50_p90": r["pair_ms_p10_p50_p90"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic: %d^3 real field, random-phase k^-5/3 spectrum (|k|<=%d), unit RMS, seed 3" % (
            n, n // 3),
        "config": {"workload": "3D r2c+c2r pair %dx%dx%d %s (r2c x->X, c2r X->y with work), natural-order "
                               "n0 x n1 x %d spectrum" % (n, n, n, head, n // 2 + 1),
                   "shape": list(shape), "parallelism": "single GPU"},
        "hbm_frac_alg": round(r["hbm_frac_alg"], 4),
        "hbm_frac_min": round(r["hbm_frac_min"], 4),
        "hbm_frac_swept": round(r["hbm_frac_swept"], 4),
        "hbm_frac_meas": None if r["hbm_frac_meas"] is None else round(r["hbm_frac_meas"], 4),
        "B_alg_per_pair": r["B_alg_per_pair"],
        "B_meas_per_pair": r["B_meas_per_pair"],
        "GB_s_alg": round(r["GB_s_alg"], 1),
        "gflops": round(r["gflops"], 1),
        "paper_steps": r["steps"],
        "kernels": r["kernels"],
        "roofline": r["roofline"],
        "plan": r["plan"],
        "cpu_baseline": cpu,
        "copy_GB_s": round(copy_gbs, 1),
        "batch": batch,
        "served": served,
        "ablation_transpose": ablation,
        "pruned_two_thirds": pruned,
        "autotune": tune or None,
        "sizes": sizes,
        "served_samples": served_acc,
    }
    for k in ("rel_l2_r2c", "rel_l2_c2r"):
        if k in r:
            line[k] = r[k]
    for d in dtypes[1:]:
        o = results[d]
        line[d] = {"value": round(o["pairs_s"], 2), "unit": "pairs/s", "ms_per_step": round(o["ms_per_pair"], 4),
                   "pair_ms_p10_p50_p90": o["pair_ms_p10_p50_p90"],
                   "hbm_frac_alg": round(o["hbm_frac_alg"], 4), "hbm_frac_min": round(o["hbm_frac_min"], 4),
                   "hbm_frac_swept": round(o["hbm_frac_swept"], 4),
                   "hbm_frac_meas": None if o["hbm_frac_meas"] is None else round(o["hbm_frac_meas"], 4),
                   "B_alg_per_pair": o["B_alg_per_pair"], "B_meas_per_pair": o["B_meas_per_pair"],
                   "gflops": round(o["gflops"], 1), "paper_steps": o["steps"], "kernels": o["kernels"],
                   "roofline": o["roofline"], "plan": o["plan"]}
        for k in ("rel_l2_r2c", "rel_l2_c2r"):
            if k in o:
                line[d][k] = o[k]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
