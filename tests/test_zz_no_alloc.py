"""GPU test of the allocation-free batched entry point
(fft3d_batch_submit_static): the same items through it and through
fft3d_batch_submit must give bit-identical outputs, on two calls in a row
(the second with a smaller batch, so the static array holds the first call's
task image when the second starts), with clean error bits; a
batch beyond the array's limit is refused with nothing enqueued."""
import numpy as np
import pytest

from workloads import fields
from tests.gpu_util import TOL, dev_real, host, rel_l2, rounded, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    fft3d.fft3d_init()  # batch ring and the static array's address on this device
    return fft3d


def _make(F, specs, seed0):
    """specs: (shape, dtype, direction); returns plans, inputs and two output sets."""
    import torch
    plans, rows = {}, []
    for i, (shape, dtype, d) in enumerate(specs):
        key = (shape, dtype)
        if key not in plans:
            plans[key] = F.Plan(*shape, dtype=dtype)
        p = plans[key]
        x = dev_real(rounded(fields.uniform(shape, seed0 + i), dtype), dtype)
        if d == F.FFT3D_C2R:
            inp = F.r2c(p, x)
        else:
            inp = x
        sets = []
        for _ in range(2):
            mid = F.empty_complex(p) if d == F.FFT3D_ROUNDTRIP else None
            out = F.empty_complex(p) if d == F.FFT3D_R2C else F.empty_real(p)
            work = F.empty_complex(p) if d != F.FFT3D_R2C else None
            for t in (mid, out, work):
                if t is not None:
                    t.fill_(float("nan"))
            sets.append((mid, out, work))
        rows.append((p, d, inp, sets))
    torch.cuda.synchronize()
    return plans, rows


def _items(rows, k):
    return [(p, d, inp, s[k][0], s[k][1], s[k][2]) for (p, d, inp, s) in rows]


def _same(a, b):
    import torch
    return torch.equal(a.view(torch.uint8), b.view(torch.uint8))


def _run_and_compare(F, specs, seed0):
    import torch
    plans, rows = _make(F, specs, seed0)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    say("no-alloc batch of %d items: ring" % len(rows))
    F.fft3d_batch_submit(_items(rows, 0))
    say("no-alloc batch of %d items: static" % len(rows))
    F.fft3d_batch_submit_static(_items(rows, 1), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for i, (p, d, inp, s) in enumerate(rows):
        for j in range(2):
            a, b = s[0][j], s[1][j]
            if a is None:
                continue
            if j == 2 and d == F.FFT3D_R2C:
                continue
            assert _same(a, b), (i, specs[i], j)
    return plans, rows


MIX_A = [((32, 32, 32), "f64", 2), ((48, 48, 48), "f32", 2), ((192, 192, 96), "f32", 2),
         ((64, 64, 64), "f64", 0), ((96, 96, 96), "f32", 1), ((128, 128, 128), "f64", 2),
         ((256, 256, 256), "f32", 2), ((30, 40, 50), "f64", 2), ((64, 64, 64), "f32", 2),
         ((192, 192, 96), "f64", 1), ((32, 32, 32), "f32", 0), ((96, 96, 96), "f64", 2)]
MIX_B = [((32, 32, 32), "f32", 2), ((48, 48, 48), "f64", 0), ((16, 16, 16), "f64", 1)]


def test_static_batch_matches_ring_on_two_calls(F, oracle):
    import torch
    # first call: twelve items incl. split planes (256^3) and one radix-5
    # item (which runs its own kernels after the batched launch)
    _run_and_compare(F, MIX_A, 5000)
    # second call, smaller: the array still holds the first call's image
    plans, rows = _run_and_compare(F, MIX_B, 6000)
    # and one result of the second call against the oracle
    p, d, inp, s = rows[0]
    x = host(inp).astype(np.float64)
    ref = oracle.c2r(oracle.r2c(x), 32)
    assert rel_l2(host(s[1][1]), ref) <= TOL["f32"]


def test_static_batch_limit_refused(F):
    import torch
    # 1100 ROUNDTRIP items of 8^3 make 4400 passes: beyond the 4096 the
    # array holds, so the call is refused and enqueues nothing
    p = F.Plan(8, 8, 8, dtype="f32")
    n = 1100
    x = torch.zeros((n, 8, 8, 8), dtype=torch.float32, device="cuda")
    mid = torch.zeros((n, 8, 8, 5), dtype=torch.complex64, device="cuda")
    out = torch.full((n, 8, 8, 8), 7.0, dtype=torch.float32, device="cuda")
    work = torch.zeros((n, 8, 8, 5), dtype=torch.complex64, device="cuda")
    items = [(p, F.FFT3D_ROUNDTRIP, x[i], mid[i], out[i], work[i]) for i in range(n)]
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_batch_submit_static(items)
    assert e.value.code == F.FFT3D_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # a batch within the limit on the same items runs
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    F.fft3d_batch_submit_static(items[:100], status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert bool((out[:100] == 0).all()) and bool((out[100:] == 7.0).all())
