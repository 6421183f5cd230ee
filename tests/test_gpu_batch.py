"""GPU tests of the batched form: many fields of mixed shape and dtype in one
persistent launch (ring-backed fft3d_batch_submit, and a batch handle launched
as a hipGraph or directly).

The batch runs every item with the same radix schedules as the item alone, so
each output must be bit-identical to the single-item path (fft3d_r2c /
fft3d_c2r), which the parity tests pin to the FP64 oracle; a sample of items
is also checked against the oracle directly here.
"""

import numpy as np
import pytest

from workloads import fields
from tests.gpu_util import TOL, dev_cplx, dev_real, host, rel_l2, rounded, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    fft3d.fft3d_init()  # the device's batch ring
    return fft3d


_PLANS = {}


def plan_for(F, shape, dtype):
    key = (tuple(shape), dtype)
    if key not in _PLANS:
        _PLANS[key] = F.Plan(*shape, dtype=dtype)
    return _PLANS[key]


class Item:
    """One batch item with its inputs, its batched outputs and the outputs of
    the same transform run alone."""

    def __init__(self, F, shape, dtype, direction, seed, work=True):
        import torch
        self.plan = plan_for(F, shape, dtype)
        self.is_c2r = direction == F.FFT3D_C2R
        self.shape, self.dtype, self.dir = shape, dtype, direction
        p = self.plan
        if direction == F.FFT3D_C2R:
            # a Hermitian-consistent spectrum: r2c of a field
            x = dev_real(rounded(fields.uniform(shape, seed), dtype), dtype)
            self.X0 = F.r2c(p, x)
            torch.cuda.synchronize()
            self.inp = self.X0.clone()
        else:
            self.inp = dev_real(rounded(fields.uniform(shape, seed), dtype), dtype)
        self.mid = F.empty_complex(p) if direction == F.FFT3D_ROUNDTRIP else None
        self.out = F.empty_complex(p) if direction == F.FFT3D_R2C else F.empty_real(p)
        self.work = F.empty_complex(p) if (work and direction != F.FFT3D_R2C) else None
        self._alone(F)
        self.reset()

    def _alone(self, F):
        import torch
        p = self.plan
        if self.dir == F.FFT3D_R2C:
            self.ref_out = F.r2c(p, self.inp)
            self.ref_mid = None
        elif self.dir == F.FFT3D_C2R:
            Xs = self.inp.clone()
            self.ref_out = F.c2r(p, Xs, work=F.empty_complex(p) if self.work is not None else None)
            self.ref_mid = None
        else:
            self.ref_mid = F.r2c(p, self.inp)
            Xs = self.ref_mid.clone()
            self.ref_out = F.c2r(p, Xs, work=F.empty_complex(p) if self.work is not None else None)
            if self.work is None:
                self.ref_mid = Xs  # without work the spectrum buffer ends as scratch
        torch.cuda.synchronize()

    def reset(self):
        """Poison the outputs (and restore a C2R input used as scratch)."""
        self.out.fill_(float("nan"))
        if self.mid is not None:
            self.mid.fill_(float("nan"))
        if self.is_c2r and self.work is None:
            self.inp.copy_(self.X0)

    def tuple(self):
        return (self.plan, self.dir, self.inp, self.mid, self.out, self.work)

    def check_bits(self):
        assert bool((self.out == self.ref_out).all()), "%s %s dir %d: output differs from alone" % (
            self.shape, self.dtype, self.dir)
        if self.mid is not None:
            assert bool((self.mid == self.ref_mid).all()), "%s %s: spectrum differs from alone" % (
                self.shape, self.dtype)


def _sync():
    import torch
    torch.cuda.synchronize()


def test_mixed_batch_matches_alone_and_oracle(F, oracle):
    """The 64-field mix (seed 4): every field's spectrum and round trip
    bit-identical to the field alone; one field per (shape, dtype) against
    the oracle."""
    mix = fields.batch_mix(64, seed=4)
    say("batch: 64-field mix")
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 1000 + i) for i, (s, d) in enumerate(mix)]
    F.fft3d_batch_submit([it.tuple() for it in items])
    _sync()
    for it in items:
        it.check_bits()
    seen = set()
    for it in items:
        key = (it.shape, it.dtype)
        if key in seen:
            continue
        seen.add(key)
        x = host(it.inp).astype(np.float64)
        Xo = oracle.r2c(x)
        e1 = rel_l2(host(it.mid), Xo)
        e2 = rel_l2(host(it.out), x * float(np.prod(it.shape)))
        assert e1 <= TOL[it.dtype] and e2 <= TOL[it.dtype], (key, e1, e2)


@pytest.mark.parametrize("mode", [0, 4], ids=["levels", "persistent"])
@pytest.mark.parametrize("flags", [0, 4], ids=["graph", "direct"])
def test_batch_handle_replays(F, flags, mode):
    """A batch handle launched three times (graph replays, or direct launches)
    with unrelated device work in between, in level mode (the rule) and as
    the persistent launch: every launch bit-identical to the items alone,
    status clean."""
    import torch
    mix = [((32, 32, 32), "f64"), ((48, 48, 48), "f32"), ((96, 96, 96), "f64"), ((64, 64, 64), "f32"),
           ((128, 128, 128), "f32"), ((192, 192, 96), "f64")]
    say("batch handle flags=%d mode=%d" % (flags, mode))
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 2000 + i) for i, (s, d) in enumerate(mix)]
    b = F.Batch([it.tuple() for it in items], flags, tuning={"mode": mode})
    desc = b.describe()
    assert desc["items"] == len(items) and desc["graph"] == (flags == 0)
    assert (desc["mode"] == "levels") == (mode == 0)
    assert len(desc["tasks"]) >= 4 * len(items) and desc["tickets"] > 0
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for it in items:
            it.reset()
        junk.mul_(1.0001).add_(0.5)
        b.launch()
        _sync()
        for it in items:
            it.check_bits()
        assert b.status() == 0
    b.close()


def test_directions_and_work_modes(F):
    """R2C, C2R with and without work (in place), ROUNDTRIP without work, in
    one batch; the C2R input is untouched when work is given."""
    say("batch: directions")
    R, C, T = F.FFT3D_R2C, F.FFT3D_C2R, F.FFT3D_ROUNDTRIP
    specs = [((32, 32, 32), "f64", R, True), ((48, 36, 64), "f32", C, True), ((64, 64, 64), "f64", C, False),
             ((96, 64, 32), "f32", T, False), ((12, 9, 24), "f64", T, True), ((1, 8, 16), "f32", R, True),
             ((8, 1, 8), "f64", C, True), ((1, 1, 2), "f32", T, True)]
    items = [Item(F, s, d, r, 3000 + i, work=w) for i, (s, d, r, w) in enumerate(specs)]
    F.fft3d_batch_submit([it.tuple() for it in items])
    _sync()
    for it in items:
        it.check_bits()
        if it.dir == C and it.work is not None:
            assert bool((it.inp == it.X0).all()), "C2R with work modified its input"


BIG_ALONE = [((96, 96, 96), "f64"), ((128, 128, 128), "f64"), ((192, 192, 96), "f32"), ((256, 256, 256), "f32"),
             ((8, 512, 512), "f64"), ((3, 1024, 1024), "f32"), ((1024, 2, 2), "f32"), ((2, 2048, 16), "f64"),
             ((4, 16, 4096), "f32"), ((729, 4, 6), "f64"), ((24, 256, 256), "f64")]


def test_batch_retiles_big_items_bit_identically(F):
    """Items whose own kernels are big-tier (fused big planes, wide column
    tiles) take small-tier tiles in the batch -- the split plane step,
    narrower columns -- with the same schedules: still bit-identical."""
    say("batch: retiled big items")
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 4000 + i) for i, (s, d) in enumerate(BIG_ALONE)]
    F.fft3d_batch_submit([it.tuple() for it in items])
    _sync()
    for it in items:
        it.check_bits()


@pytest.mark.parametrize("mode", ["pinned", "spread"])
@pytest.mark.parametrize("lag", [0, 1, 2, 5])
def test_ticket_orders_give_same_bits(F, lag, mode):
    """Other ticket orders (an item's passes `lag` slots apart instead of
    pass-major) and both queue modes (items pinned to XCDs, or one queue for
    all), set through the batch tuning, change only the schedule, never the
    bits."""
    mix = fields.batch_mix(12, seed=7)
    say("batch: lag %s mode %s" % (lag, mode))
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 5000 + i) for i, (s, d) in enumerate(mix)]
    b = F.Batch([it.tuple() for it in items], tuning={"mode": 1 if mode == "pinned" else 2, "lag": lag})
    assert b.describe()["mode"] == mode
    b.launch()
    _sync()
    for it in items:
        it.check_bits()
    assert b.status() == 0


@pytest.mark.parametrize("widen,wg,mode", [(2, 0, 0), (2, 0, 4), (1, 1, 4), (2, 1, 4)])
def test_batch_tile_shapes_give_same_bits(F, widen, wg, mode):
    """The plans' own tile shapes instead of widened ones (level mode and
    persistent), and one workgroup per CU (persistent): same bits."""
    mix = fields.batch_mix(10, seed=17)
    say("batch: widen %d wg_per_cu %d mode %d" % (widen, wg, mode))
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 5500 + i) for i, (s, d) in enumerate(mix)]
    b = F.Batch([it.tuple() for it in items], flags=F.FFT3D_BATCH_DIRECT,
                tuning={"widen": widen, "wg_per_cu": wg, "mode": mode})
    b.launch()
    _sync()
    for it in items:
        it.check_bits()
    assert b.status() == 0


@pytest.mark.parametrize("flags", [0, 4], ids=["graph", "direct"])
def test_level_mode_gives_same_bits(F, flags):
    """Level mode (batch tuning mode 3: one launch per pass level, tile kind
    and dtype, in one graph or launched directly): the 64-field mix, the
    retiled big items and every direction and work mode, bit-identical to the
    items alone, three launches in a row with unrelated device work between
    them; status 0."""
    import torch
    R, C, T = F.FFT3D_R2C, F.FFT3D_C2R, F.FFT3D_ROUNDTRIP
    specs = [(s, d, T, True) for s, d in fields.batch_mix(64, seed=4)]
    specs += [(s, d, T, True) for s, d in BIG_ALONE[:6]]
    # FP32 lines of radix <= 8 schedules (512 = 8*8*8, 64 = 8*8) run on the
    # fine column tier alone and on the 512-thread small tier here: same bits
    specs += [((8, 512, 512), "f32", T, True), ((512, 8, 64), "f32", T, True)]
    specs += [((32, 32, 32), "f64", R, True), ((48, 36, 64), "f32", C, True), ((64, 64, 64), "f64", C, False),
              ((96, 64, 32), "f32", T, False), ((12, 9, 24), "f64", T, True), ((1, 8, 16), "f32", R, True),
              ((8, 1, 8), "f64", C, True), ((1, 1, 2), "f32", T, True)]
    say("batch: level mode flags=%d, %d items" % (flags, len(specs)))
    items = [Item(F, s, d, r, 9100 + i, work=w) for i, (s, d, r, w) in enumerate(specs)]
    b = F.Batch([it.tuple() for it in items], flags=flags, tuning={"mode": 3})
    desc = b.describe()
    assert desc["mode"] == "levels" and desc["graph"] == (flags == 0)
    launches = desc["launches"]
    assert launches and sum(L[2] for L in launches) == len(desc["tasks"])
    assert sum(L[3] for L in launches) == desc["tickets"]
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for it in items:
            it.reset()
        junk.mul_(1.0001).add_(0.5)
        b.launch()
        _sync()
        for it in items:
            it.check_bits()
            if it.dir == C and it.work is not None:
                assert bool((it.inp == it.X0).all()), "C2R with work modified its input"
        assert b.status() == 0
    b.close()


def test_wait_error_path_ends_the_launch(F):
    """The persistent launch (mode 4) with dependency waits that give up at
    once (batch tuning spin_limit < 0, no poll): every second pass of an item
    fails its wait, its tiles are skipped, and the launch still ends with
    error bit 1 -- twice in a row on the same handle (the last workgroup
    clears the counters either way).  A handle with the rule then computes
    the same items correctly."""
    mix = fields.batch_mix(8, seed=23)
    say("batch: wait error path")
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 8300 + i) for i, (s, d) in enumerate(mix)]
    for flags in (0, F.FFT3D_BATCH_DIRECT):
        b = F.Batch([it.tuple() for it in items], flags=flags, tuning={"spin_limit": -1, "mode": 4})
        for _ in range(2):
            b.launch()
            _sync()
            assert b.status() & 1
    for it in items:
        it.reset()
    ok = F.Batch([it.tuple() for it in items])
    ok.launch()
    _sync()
    assert ok.status() == 0
    for it in items:
        it.check_bits()


def test_sequential_flag_matches(F):
    mix = fields.batch_mix(6, seed=8)
    say("batch: sequential flag")
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 6000 + i) for i, (s, d) in enumerate(mix)]
    F.fft3d_batch_submit_ex([it.tuple() for it in items], F.FFT3D_BATCH_SEQUENTIAL)
    _sync()
    for it in items:
        it.check_bits()


def test_ring_reuse_and_streams(F):
    """More submits than ring slots, alternating two streams: the staging ring
    wraps (waiting on its slots' events) and every result stays right."""
    import torch
    say("batch: ring wrap, two streams")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rounds = []
    for r in range(20):
        s, d = fields.BATCH_SHAPES[r % 3], ("f32", "f64")[r % 2]
        items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 7000 + 10 * r + j) for j in range(2)]
        rounds.append(items)
    _sync()
    for r, items in enumerate(rounds):
        F.fft3d_batch_submit([it.tuple() for it in items], stream=streams[r % 2])
    _sync()
    for items in rounds:
        for it in items:
            it.check_bits()


def test_many_items_split_into_launches(F):
    """More items than one ring slot holds (about 680): the submit splits them
    into several launches on the stream."""
    say("batch: 700 tiny items")
    shapes = [(2, 3, 4), (3, 4, 6), (4, 6, 2), (1, 8, 16), (8, 1, 8)]
    items = [Item(F, shapes[i % 5], ("f32", "f64")[i % 2], F.FFT3D_ROUNDTRIP, 8000 + i) for i in range(700)]
    F.fft3d_batch_submit([it.tuple() for it in items])
    _sync()
    for it in items:
        it.check_bits()


def test_batch_determinism(F):
    mix = fields.batch_mix(16, seed=9)
    say("batch: determinism")
    items = [Item(F, s, d, F.FFT3D_ROUNDTRIP, 9000 + i) for i, (s, d) in enumerate(mix)]
    first = None
    for rep in range(5):
        for it in items:
            it.reset()
        F.fft3d_batch_submit([it.tuple() for it in items])
        _sync()
        outs = [host(it.out).copy() for it in items]
        if first is None:
            first = outs
        else:
            for a, b in zip(first, outs):
                assert np.array_equal(a, b)


def test_batch_validation(F):
    """Overlapping written buffers across items, a bad direction, an empty
    handle: rejected before anything is enqueued."""
    import torch
    say("batch: validation")
    p = F.Plan(16, 16, 16, dtype="f32")
    x = dev_real(fields.uniform((16, 16, 16), 1), "f32")
    X = F.empty_complex(p)
    X.fill_(7.0)
    X2 = F.empty_complex(p)
    # two items writing the same spectrum
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_batch_submit([(p, F.FFT3D_R2C, x, None, X, None), (p, F.FFT3D_R2C, x, None, X, None)])
    assert e.value.code == F.FFT3D_ERR_INVALID_ARG and "concurrently" in str(e.value)
    _sync()
    assert bool((X == 7.0).all()), "a rejected batch enqueued work"
    # one item reads what another writes
    y = F.empty_real(p)
    with pytest.raises(F.Fft3dError):
        F.fft3d_batch_submit([(p, F.FFT3D_R2C, x, None, X, None), (p, F.FFT3D_C2R, X, None, y, X2)])
    # shared read-only input is fine
    X3 = F.empty_complex(p)
    F.fft3d_batch_submit([(p, F.FFT3D_R2C, x, None, X2, None), (p, F.FFT3D_R2C, x, None, X3, None)])
    _sync()
    assert bool((X2 == X3).all())
    with pytest.raises(F.Fft3dError):
        F.fft3d_batch_submit([(p, 7, x, None, X, None)])
    F.fft3d_batch_submit([])  # nothing to do
    with pytest.raises(F.Fft3dError):
        F.Batch([])
    with pytest.raises(F.Fft3dError):
        F.fft3d_batch_submit_ex([(p, F.FFT3D_R2C, x, None, X, None)], 64)
    torch.cuda.synchronize()
