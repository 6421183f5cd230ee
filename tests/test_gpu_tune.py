"""GPU tests of the autotuner and of tuned plans.

A tuning changes only how the passes are cut into launches (plane step
kind, tile shapes, XCD grouping, walk order) -- the results must be bit for
bit those of the rule plan -- or the radix schedule, which changes the
rounding only: those plans are checked against the FP64 oracle at the
acceptance bounds.  The tuner itself must return a tuning that makes a valid
plan, keep it in the table (lookup, save, load), and the batch tuner a
launch shape that gives the same bits."""
import numpy as np
import pytest

from workloads import fields
from tests.gpu_util import TOL, dev_cplx, dev_real, host, oracle_threads, rel_l2, rounded, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    fft3d.fft3d_init()
    return fft3d


def pair(F, plan, x, S):
    """r2c of x, and c2r (with work) of the spectrum S; both on the device."""
    import torch
    X = F.r2c(plan, x)
    y = F.c2r(plan, S.clone(), work=F.empty_complex(plan))
    torch.cuda.synchronize()
    return X, y


def same_bits(a, b):
    import torch
    return torch.equal(a.view(torch.uint8), b.view(torch.uint8))


TILE_TUNINGS = {
    (64, 64, 64): [dict(plane=2), dict(plane=2, rows_rpw=4, n1_w=4), dict(n0_w=4, n0_group=1), dict(walk=64 + 63)],
    (256, 256, 256): [dict(rows_rpw=4), dict(rows_rpw=32), dict(rows_rpw_inv=4), dict(rows_rpw=8, rows_rpw_inv=24),
                      dict(n1_w=4), dict(n1_w=32), dict(n0_w=8, n0_group=2),
                      dict(n0_w=32, n0_group=1), dict(walk=64), dict(walk=64 + 63),
                      dict(plane=3), dict(plane=3, coop_lag=1), dict(plane=3, coop_lag=16, coop_rpw=4, coop_w=4)],
    (96, 128, 384): [dict(rows_rpw=6), dict(rows_rpw_inv=6), dict(plane=3, coop_lag=5), dict(n0_w=32, n0_group=3)],
}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", list(TILE_TUNINGS))
def test_tile_tunings_bit_identical_to_rule(F, oracle, shape, dtype):
    x64 = fields.uniform(shape, seed=71)
    x = dev_real(rounded(x64, dtype), dtype)
    rule = F.Plan(*shape, dtype=dtype)
    S = F.r2c(rule, x)
    X0, y0 = pair(F, rule, x, S)
    # the rule plan itself against the oracle once
    assert rel_l2(host(X0), oracle.r2c(rounded(x64, dtype))) <= TOL[dtype]
    for t in TILE_TUNINGS[shape]:
        say("tile tuning %s %s %s" % (shape, dtype, t))
        p = F.Plan(*shape, dtype=dtype, tuning=t)
        X, y = pair(F, p, x, S)
        assert same_bits(X, X0), t
        assert same_bits(y, y0), t


# Wide column tiles (1024-long columns) walked by the persistent loop that
# loads a tile ahead (the rule) against one tile per workgroup: more tiles
# than workgroups (each workgroup walks several), a ragged last tile, n0
# passes over one block and n1 passes over several planes.
PIPE_SHAPES = [(1024, 98, 84), (10, 1024, 1024), (1024, 3, 18)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", PIPE_SHAPES)
def test_pipelined_wide_columns(F, oracle, shape, dtype):
    say("pipelined wide columns %s %s" % (shape, dtype))
    x64 = rounded(fields.uniform(shape, seed=83), dtype)
    rule = F.Plan(*shape, dtype=dtype)
    plain = F.Plan(*shape, dtype=dtype, tuning=dict(cols_pipe=1))
    d, dp = rule.describe(), plain.describe()
    for desc, pipe in ((d, True), (dp, False)):
        passes = [desc["n0_pass"]] + ([desc["plane"]["n1_pass"]] if "n1_pass" in desc["plane"] else [])
        wide = [c for c in passes if c["tier"] == "wide"]
        assert wide and all(c["pipe"] == pipe for c in wide)
    x = dev_real(x64, dtype)
    Xo = oracle.r2c(x64, threads=oracle_threads())
    S = dev_cplx(rounded(Xo, dtype), dtype)
    X0, y0 = pair(F, rule, x, S)
    X1, y1 = pair(F, plain, x, S)
    assert same_bits(X0, X1) and same_bits(y0, y1)
    assert rel_l2(host(X0), Xo) <= TOL[dtype]
    assert rel_l2(host(y0), oracle.c2r(rounded(Xo, dtype), shape[2], threads=oracle_threads())) <= TOL[dtype]


def test_pipelined_wide_columns_four_stages(F, oracle):
    # 2048-long columns on the wide tier (8 columns a tile, ragged last tile)
    # with a four-stage schedule: twiddles of three later stages in LDS
    shape, t = (2048, 6, 10), dict(n0_w=8, radix=[[8, 8, 8, 4], [], []])
    say("pipelined wide columns %s %s" % (shape, t))
    x64 = rounded(fields.uniform(shape, seed=85), "f32")
    a = F.Plan(*shape, dtype="f32", tuning=t)
    b = F.Plan(*shape, dtype="f32", tuning=dict(t, cols_pipe=1))
    assert a.describe()["n0_pass"]["pipe"] and not b.describe()["n0_pass"]["pipe"]
    x = dev_real(x64, "f32")
    Xo = oracle.r2c(x64)
    S = dev_cplx(rounded(Xo, "f32"), "f32")
    X0, y0 = pair(F, a, x, S)
    X1, y1 = pair(F, b, x, S)
    assert same_bits(X0, X1) and same_bits(y0, y1)
    assert rel_l2(host(X0), Xo) <= TOL["f32"]
    assert rel_l2(host(y0), oracle.c2r(rounded(Xo, "f32"), shape[2])) <= TOL["f32"]


RADIX_TUNINGS = [
    ((512, 64, 256), dict(radix=[[16, 16, 2], [], []])),
    ((512, 64, 256), dict(radix=[[2, 16, 16], [4, 16], [8, 16]])),
    ((64, 96, 192), dict(radix=[[4, 16], [3, 4, 8], [3, 8, 4]])),
    ((256, 256, 256), dict(radix=[[4, 4, 16], [16, 4, 4], [2, 4, 16]], plane=3, coop_lag=3)),
    ((40, 49, 100), dict(radix=[[8, 5], [7, 7], [5, 2, 5]])),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", range(len(RADIX_TUNINGS)))
def test_radix_tunings_match_oracle(F, oracle, case, dtype):
    shape, t = RADIX_TUNINGS[case]
    say("radix tuning %s %s %s" % (shape, dtype, t))
    x64 = rounded(fields.uniform(shape, seed=73 + case), dtype)
    p = F.Plan(*shape, dtype=dtype, tuning=t)
    d = p.describe()
    for a, key in enumerate(("n0", "n1", "n2_half")):
        if t["radix"][a]:
            assert d["schedules"][key]["radices"] == t["radix"][a]
    x = dev_real(x64, dtype)
    Xo = oracle.r2c(x64)
    S = dev_cplx(rounded(Xo, dtype), dtype)
    X, y = pair(F, p, x, S)
    assert rel_l2(host(X), Xo) <= TOL[dtype]
    yo = oracle.c2r(rounded(Xo, dtype), shape[2])
    assert rel_l2(host(y), yo) <= TOL[dtype]


@pytest.mark.parametrize("shape,dtype", [((64, 64, 64), "f32"), ((256, 256, 256), "f32"), ((128, 128, 128), "f64")])
def test_autotune_table_and_tuned_plan(F, oracle, tmp_path, shape, dtype):
    say("autotune %s %s" % (shape, dtype))
    best, report = F.autotune(shape, dtype, effort=0)
    assert report["shape"] == list(shape) and report["dtype"] == dtype
    assert report["pair_ms_rule"] > 0 and len(report["candidates"]) > 3
    assert report["best"] == best
    if report["kept"] == "tuned":
        assert report["pair_ms_tuned"] < report["pair_ms_rule"]
    # the table has it; a tuned plan takes it
    assert F.fft3d_tune_lookup(*shape, dtype=dtype) == best
    p = F.Plan(*shape, dtype=dtype, tuned=True)
    assert p.describe()["tuning"] == best
    # round trip through a file
    path = tmp_path / "tune.json"
    F.fft3d_tune_save(str(path))
    F.fft3d_tune_load(str(path))
    assert F.fft3d_tune_lookup(*shape, dtype=dtype) == best
    # the tuned plan against the oracle
    x64 = rounded(fields.uniform(shape, seed=77), dtype)
    x = dev_real(x64, dtype)
    Xo = oracle.r2c(x64)
    X, y = pair(F, p, x, dev_cplx(rounded(Xo, dtype), dtype))
    assert rel_l2(host(X), Xo) <= TOL[dtype]
    assert rel_l2(host(y), oracle.c2r(rounded(Xo, dtype), shape[2])) <= TOL[dtype]


def test_autotune_times_the_persistent_column_loop(F, oracle):
    # a shape with wide column passes: the search times the loop against one
    # tile per workgroup, and whichever it keeps matches the oracle
    shape = (1024, 16, 18)
    say("autotune with wide column passes %s" % (shape,))
    best, report = F.autotune(shape, "f32", effort=0)
    stages = [c for c in report["candidates"] if c["stage"] == "cols_pipe"]
    # the stage runs when the tiling chosen before it has a persistent pass
    # (the earlier stages may have moved the n0 pass off the wide tier)
    d = F.Plan(*shape, dtype="f32", host_only=True, tuning=dict(best, cols_pipe=0)).describe()
    say("tuned %s, persistent n0 pass before the stage: %s" % (best, d["n0_pass"]["pipe"]))
    if d["n0_pass"]["pipe"]:
        assert len(stages) == 2 and all(c["ms"] and c["ms"] > 0 for c in stages)
    else:
        assert not stages and best["cols_pipe"] == 0
    assert best["cols_pipe"] in (0, 1)
    p = F.Plan(*shape, dtype="f32", tuning=best)
    x64 = rounded(fields.uniform(shape, seed=87), "f32")
    Xo = oracle.r2c(x64)
    X, y = pair(F, p, dev_real(x64, "f32"), dev_cplx(rounded(Xo, "f32"), "f32"))
    assert rel_l2(host(X), Xo) <= TOL["f32"]
    assert rel_l2(host(y), oracle.c2r(rounded(Xo, "f32"), shape[2])) <= TOL["f32"]


def test_batch_autotune_gives_same_bits(F):
    import torch
    mix = fields.batch_mix(8, seed=79)
    say("batch autotune over %d items" % len(mix))
    plans, rows = {}, []
    for i, (shape, dtype) in enumerate(mix):
        if (shape, dtype) not in plans:
            plans[(shape, dtype)] = F.Plan(*shape, dtype=dtype)
        p = plans[(shape, dtype)]
        x = dev_real(rounded(fields.uniform(shape, 7900 + i), dtype), dtype)
        rows.append((p, x, F.empty_complex(p), F.empty_real(p), F.empty_complex(p)))
    items = [(p, F.FFT3D_ROUNDTRIP, x, m, o, w) for (p, x, m, o, w) in rows]
    best, report = F.fft3d_batch_autotune(items, effort=0)
    assert report["ms_rule"] > 0 and report["best"] == best
    assert len(report["candidates"]) >= 10
    # the rule batch and the tuned batch give the same bits
    F.Batch(items).launch()
    torch.cuda.synchronize()
    ref = [(m.clone(), o.clone()) for (p, x, m, o, w) in rows]
    for (p, x, m, o, w) in rows:
        m.fill_(float("nan"))
        o.fill_(float("nan"))
    b = F.Batch(items, tuning=best)
    b.launch()
    torch.cuda.synchronize()
    assert b.status() == 0
    for (p, x, m, o, w), (m0, o0) in zip(rows, ref):
        assert same_bits(m, m0) and same_bits(o, o0)
