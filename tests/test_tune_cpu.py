"""CPU tests of the tuning interface: which tunings a plan accepts and how
they show in its description (host-only plans), and the tuning table's JSON
file (load, save, refusals).  No kernel runs here."""
import json
import os

import pytest


@pytest.fixture(scope="module")
def F():
    from paper_1406_5597_amd import fft3d
    return fft3d


def desc(F, shape, dtype="f32", **tuning):
    return F.Plan(*shape, dtype=dtype, host_only=True, tuning=tuning).describe()


def test_zero_tuning_is_the_rule(F):
    for shape, dtype in [((512, 512, 512), "f32"), ((64, 64, 64), "f64"), ((30, 42, 50), "f32"), ((16, 128, 243), "f64")]:
        a = F.Plan(*shape, dtype=dtype, host_only=True).describe()
        b = desc(F, shape, dtype)
        assert b["tuning"] is not None and a["tuning"] is None
        a.pop("tuning"), b.pop("tuning")
        assert a == b


def test_tile_fields_take_effect(F):
    d = desc(F, (512, 512, 512), rows_rpw=8, n1_w=8, n0_w=32, n0_group=4, walk=64 + 5)
    assert d["plane"]["kind"] == "split" and d["plane"]["rows_per_wg"] == 8
    assert d["plane"]["n1_pass"]["W"] == 8 and d["n0_pass"]["W"] == 32
    assert d["n0_group"] == 4 and d["rev"] == 5
    assert d["tuning"]["rows_rpw"] == 8 and d["tuning"]["walk"] == 69
    # 1024-long n0 columns: 16 wide take the wide tier (128 KB), 32 wide fit no tier
    d = desc(F, (1024, 64, 64), n0_w=16)
    assert d["n0_pass"]["W"] == 16 and d["n0_pass"]["tier"] == "wide"
    with pytest.raises(F.Fft3dError):
        desc(F, (1024, 64, 64), n0_w=32)


def test_rows_tiles_per_direction(F):
    # FP32, even n2: the forward rows tile within 40 KB of LDS (four
    # workgroups a CU), the inverse within 48 KB (three)
    d = F.Plan(512, 512, 512, dtype="f32", host_only=True).describe()["plane"]
    assert d["rows_per_wg"] == 16 and d["lds"] <= 40 * 1024 and d["grid"] == 512 * 512 // 16
    assert d["rows_per_wg_inv"] == 20 and 40 * 1024 < d["lds_inv"] <= 48 * 1024
    for shape, dtype in [((512, 512, 512), "f64"), ((16, 128, 243), "f32")]:
        d = F.Plan(*shape, dtype=dtype, host_only=True).describe()["plane"]
        assert d["rows_per_wg"] == d["rows_per_wg_inv"] and d["lds"] == d["lds_inv"]
    d = desc(F, (512, 512, 512), rows_rpw_inv=8)
    assert d["plane"]["rows_per_wg"] == 16 and d["plane"]["rows_per_wg_inv"] == 8
    assert d["plane"]["grid_inv"] == 512 * 512 // 8 and d["tuning"]["rows_rpw_inv"] == 8
    d = desc(F, (512, 512, 512), rows_rpw=12)
    assert d["plane"]["rows_per_wg"] == 12 and d["plane"]["rows_per_wg_inv"] == 20


def test_fine_column_tier(F):
    # FP32 small column tiles of radix <= 8 schedules take the fine tier
    d = F.Plan(512, 512, 512, dtype="f32", host_only=True).describe()
    assert d["schedules"]["n0"]["radices"] == [8, 8, 8]
    assert d["n0_pass"]["tier"] == "fine" and d["plane"]["n1_pass"]["tier"] == "fine"
    assert d["n0_pass"]["lds"] == 512 * 16 * 8
    d = F.Plan(512, 512, 512, dtype="f64", host_only=True).describe()
    assert d["n0_pass"]["tier"] == "small" and d["plane"]["n1_pass"]["tier"] == "small"
    d = desc(F, (512, 512, 512), radix=[[16, 16, 2], [], []])
    assert d["n0_pass"]["tier"] == "small" and d["plane"]["n1_pass"]["tier"] == "fine"
    d = F.Plan(256, 256, 256, dtype="f32", host_only=True).describe()
    assert d["schedules"]["n0"]["radices"] == [16, 16] and d["n0_pass"]["tier"] == "small"
    assert desc(F, (1024, 64, 64), n0_w=16)["n0_pass"]["tier"] == "wide"


def test_pipelined_wide_column_passes(F):
    # wide tiles of schedules with a radix-16/8 first stage and radix <= 8
    # after it walk their tiles in a persistent loop by rule; cols_pipe=1
    # gives one tile per workgroup
    for dt in ("f32", "f64"):
        d = F.Plan(1024, 1024, 1024, dtype=dt, host_only=True).describe()
        assert d["schedules"]["n0"]["radices"] == [16, 8, 8]
        for c in (d["n0_pass"], d["plane"]["n1_pass"]):
            assert c["tier"] == "wide" and c["pipe"] is True
        d = desc(F, (1024, 1024, 1024), dtype=dt, cols_pipe=1)
        assert not d["n0_pass"]["pipe"] and not d["plane"]["n1_pass"]["pipe"] and d["tuning"]["cols_pipe"] == 1
    # a later radix-16 stage, or a tier other than wide, keeps one tile per workgroup
    assert not desc(F, (1024, 64, 64), radix=[[8, 8, 16], [], []])["n0_pass"]["pipe"]
    assert not F.Plan(768, 4, 4, dtype="f32", host_only=True).describe()["n0_pass"]["pipe"]
    d = F.Plan(512, 512, 512, dtype="f32", host_only=True).describe()
    assert not d["n0_pass"]["pipe"] and not d["plane"]["n1_pass"]["pipe"]
    # the tile and the later stages' twiddles must fit LDS together: 128 KB +
    # 2040 FP32 twiddles (16 KB) do, 128 KB + 4088 FP64 twiddles (64 KB) do not
    d = desc(F, (2048, 4, 4), n0_w=8, radix=[[8, 8, 8, 4], [], []])
    assert d["n0_pass"]["tier"] == "wide" and d["n0_pass"]["pipe"]
    d = desc(F, (4096, 4, 4), dtype="f64", n0_w=2, radix=[[8, 8, 8, 8], [], []])
    assert d["n0_pass"]["tier"] == "wide" and not d["n0_pass"]["pipe"]


def test_plane_kinds(F):
    assert desc(F, (512, 512, 512), plane=F.FFT3D_TUNE_COOP, coop_lag=16, coop_rpw=10, coop_w=8)["plane"]["coop"] == {
        "row_tasks": 52, "col_tasks": 33, "rows_per_task": 10, "cols_per_task": 8, "lag": 16, "grid": 0,
        "lds": 32768, "slots": 0}
    # a plane that fits LDS: fused by rule, split on request
    assert desc(F, (64, 64, 64))["plane"]["kind"] == "fused"
    d = desc(F, (64, 64, 64), plane=F.FFT3D_TUNE_SPLIT, n1_w=16)
    assert d["plane"]["kind"] == "split" and d["plane"]["n1_pass"]["W"] == 16
    assert d["r2c_passes"] == [0, 1, 2] and d["c2r_passes"] == [3, 4, 5]


def test_radix_schedules(F):
    d = desc(F, (512, 96, 512), radix=[[16, 16, 2], [3, 8, 4], [4, 4, 16]])
    assert d["schedules"]["n0"]["radices"] == [16, 16, 2]
    assert d["schedules"]["n1"]["radices"] == [3, 8, 4]
    assert d["schedules"]["n2_half"]["radices"] == [4, 4, 16]
    # radix 5 / 7 lists select the kernels built with those stages
    d = desc(F, (40, 49, 50), radix=[[5, 8], [7, 7], [5, 5]])
    assert d["radix57"] is True and d["schedules"]["n0"]["radices"] == [5, 8]


@pytest.mark.parametrize("tuning,needle", [
    (dict(plane=1), "FUSED"), (dict(plane=4), "plane must be"), (dict(rows_rpw=100), "rows_rpw"),
    (dict(rows_rpw=-1), "rows_rpw"), (dict(rows_rpw_inv=100), "rows_rpw_inv"), (dict(rows_rpw_inv=-3), "rows_rpw_inv"),
    (dict(n1_w=3), "n1_w"), (dict(n1_w=128), "n1_w"), (dict(n0_w=12), "n0_w"),
    (dict(n0_group=-2), "n0_group"), (dict(walk=5), "walk"), (dict(walk=200), "walk"),
    (dict(coop_lag=4), "coop_"), (dict(plane=3, coop_lag=300), "coop_lag"), (dict(plane=3, coop_rpw=21), "coop_rpw"),
    (dict(plane=3, coop_w=3), "coop_w"), (dict(radix=[[16, 16, 4], [], []]), "radix[0]"),
    (dict(radix=[[], [6, 64, 1], []]), "radix[1]"), (dict(radix=[[], [], [32, 8]]), "radix[2]"),
    (dict(cols_pipe=3), "cols_pipe"), (dict(cols_pipe=-1), "cols_pipe"),
])
def test_tunings_refused(F, tuning, needle):
    with pytest.raises(F.Fft3dError) as e:
        F.Plan(512, 512, 512, dtype="f32", host_only=True, tuning=tuning)
    assert e.value.code == F.FFT3D_ERR_INVALID_ARG and needle in str(e.value)


def test_fused_plans_refuse_split_fields(F):
    with pytest.raises(F.Fft3dError):
        F.Plan(64, 64, 64, dtype="f32", host_only=True, tuning=dict(rows_rpw=4))
    with pytest.raises(F.Fft3dError):
        F.Plan(64, 64, 64, dtype="f32", host_only=True, tuning=dict(rows_rpw_inv=4))
    with pytest.raises(F.Fft3dError):  # radix-5/7 or odd n2: no cooperative step
        F.Plan(40, 250, 256, dtype="f32", host_only=True, tuning=dict(plane=3))


def test_table_file_round_trip(F, tmp_path):
    src = {"version": 1, "entries": [
        {"arch": "gfx950", "shape": [512, 512, 512], "dtype": "f32", "pair_ms_rule": 1.38, "pair_ms_tuned": 1.2,
         "tuning": {"plane": 3, "coop_lag": 16, "n0_w": 32, "n0_group": 4, "walk": 64,
                    "radix": [[16, 16, 2], [], [16, 16]]}},
        {"arch": "gfx950", "shape": [64, 64, 64], "dtype": "f64", "tuning": {"plane": 2}},
    ]}
    a = tmp_path / "a.json"
    a.write_text(json.dumps(src))
    F.fft3d_tune_load(str(a))
    b = tmp_path / "b.json"
    F.fft3d_tune_save(str(b))
    out = json.loads(b.read_text())
    assert out["version"] == 1
    got = {(e["arch"], tuple(e["shape"]), e["dtype"]): e for e in out["entries"]}
    e = got[("gfx950", (512, 512, 512), "f32")]
    assert e["tuning"]["plane"] == 3 and e["tuning"]["coop_lag"] == 16 and e["tuning"]["n0_w"] == 32
    assert e["tuning"]["radix"] == [[16, 16, 2], [], [16, 16]] and e["pair_ms_tuned"] == pytest.approx(1.2)
    assert got[("gfx950", (64, 64, 64), "f64")]["tuning"]["plane"] == 2
    # the saved file loads again
    F.fft3d_tune_load(str(b))


@pytest.mark.parametrize("text", [
    "", "{", "[]", '{"version": 2, "entries": []}', '{"version": 1}',
    '{"version": 1, "entries": [{"arch": "gfx950", "shape": [8, 8], "dtype": "f32", "tuning": {}}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "shape": [8, 8, 8], "dtype": "f16", "tuning": {}}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "shape": [512, 512, 512], "dtype": "f32", '
    '"tuning": {"rows_rpw": 1000}}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "shape": [8, 8, 8], "dtype": "f32", "tuning": {"walk": 1.5}}]}',
])
def test_bad_table_files_refused(F, tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_tune_load(str(p))
    assert e.value.code == F.FFT3D_ERR_INVALID_ARG
    with pytest.raises(F.Fft3dError):
        F.fft3d_tune_load(str(tmp_path / "missing.json"))


def test_library_reads_no_environment():
    """Tile shapes come from the plan's rule or its tuning, never from
    environment variables."""
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1406_5597_amd", "csrc")
    for f in os.listdir(root):
        src = open(os.path.join(root, f)).read()
        assert "getenv" not in src, f
