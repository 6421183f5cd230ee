"""GPU parity for odd n2 (two real rows per complex line of length n2),
against the FP64 oracle: tiles with an odd number of rows, single-row
arrays, rows long enough for the big tier, radix-3/5/7 row lengths; the
c2r definition on a non-Hermitian half spectrum; and the transpose-based and
batched entry points bit for bit against the plain transforms."""
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


SHAPES = [(2, 3, 1), (1, 1, 3), (1, 1, 5), (1, 3, 9), (4, 6, 9), (3, 5, 7), (8, 12, 15), (5, 16, 27),
          (32, 32, 27), (6, 64, 125), (16, 128, 243), (3, 24, 2187), (2, 2, 6561), (1, 3, 7203)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_odd_n2_match_oracle(F, oracle, shape, dtype):
    say("odd n2 parity %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=27), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    assert plan.half_shape == (shape[0], shape[1], shape[2] // 2 + 1)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    Xo = oracle.r2c(x)
    assert rel_l2(host(X), Xo) <= TOL[dtype], rel_l2(host(X), Xo)
    S = rounded(Xo, dtype)
    Sd = dev_cplx(S, dtype)
    S_before = Sd.clone()
    y = F.c2r(plan, Sd, work=F.empty_complex(plan))
    yo = oracle.c2r(S, shape[2])
    assert rel_l2(host(y), yo) <= TOL[dtype]
    assert bool((Sd == S_before).all())
    y2 = F.c2r(plan, Sd)  # in place
    assert rel_l2(host(y2), yo) <= TOL[dtype]
    y3 = F.c2r(plan, X)
    assert rel_l2(host(y3), x * np.prod(shape)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_odd_n2_c2r_non_hermitian_follows_definition(F, oracle, dtype):
    """Arbitrary half spectrum: the imaginary part of each row's DC bin (after
    the n0/n1 passes) is dropped; there is no Nyquist bin for odd n2."""
    shape = (6, 8, 15)
    say("odd n2 non-hermitian %s" % dtype)
    rng = np.random.default_rng(6)
    h = shape[2] // 2 + 1
    S = rounded(rng.standard_normal((6, 8, h)) + 1j * rng.standard_normal((6, 8, h)), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    y = host(F.c2r(plan, dev_cplx(S, dtype), work=F.empty_complex(plan)))
    assert rel_l2(y, oracle.c2r_direct(S, shape[2])) <= TOL[dtype]
    S2 = S.copy()
    S2[0, 0, 0] += 3j
    y2 = host(F.c2r(plan, dev_cplx(S2, dtype), work=F.empty_complex(plan)))
    assert rel_l2(y2, y) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_odd_n2_single_modes_exact_index(F, dtype):
    import torch
    shape = (12, 10, 21)
    n0, n1, n2 = shape
    say("odd n2 single modes %s" % dtype)
    plan = F.Plan(*shape, dtype=dtype)
    j0, j1, j2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    for m in [(0, 0, 10), (3, 4, 1), (-5, 2, 7), (1, 0, 0), (0, 0, 0)]:
        x = np.cos(2 * np.pi * (m[0] * j0 / n0 + m[1] * j1 / n1 + m[2] * j2 / n2))
        X = host(F.r2c(plan, dev_real(rounded(x, dtype), dtype)))
        torch.cuda.synchronize()
        big = np.argwhere(np.abs(X) > 0.25 * x.size)
        want = {(m[0] % n0, m[1] % n1, m[2])}
        if m[2] == 0:
            want.add(((-m[0]) % n0, (-m[1]) % n1, 0))
        assert {tuple(v) for v in big} == want, (m, big)


def test_odd_n2_other_entry_points(F):
    import torch
    say("odd n2 transposed / batch / pruned")
    shape = (20, 24, 45)
    n0, n1, n2 = shape
    plan = F.Plan(*shape, dtype="f32", coop_plane=True)
    assert plan.describe()["plane"]["kind"] == "split"
    xd = dev_real(fields.uniform(shape, 4), "f32")
    X = F.r2c(plan, xd)
    Xt = torch.empty((n1, n0, n2 // 2 + 1), dtype=X.dtype, device="cuda")
    work = F.empty_complex(plan)
    F.fft3d_r2c_transposed(plan, xd, Xt, work)
    torch.cuda.synchronize()
    assert bool((Xt == X.permute(1, 0, 2)).all())
    y_free = F.c2r(plan, X.clone(), work=F.empty_complex(plan))
    y = F.empty_real(plan)
    F.fft3d_c2r_transposed(plan, Xt, y, work)
    torch.cuda.synchronize()
    assert bool((y == y_free).all())
    # batch: odd-n2 items beside batchable ones, each bit for bit as alone
    p_even = F.Plan(32, 32, 32, dtype="f64")
    x_even = dev_real(fields.uniform((32, 32, 32), 5), "f64")
    X_even = F.r2c(p_even, x_even)
    items = [(plan, F.FFT3D_ROUNDTRIP, xd, F.empty_complex(plan), F.empty_real(plan), F.empty_complex(plan)),
             (p_even, F.FFT3D_R2C, x_even, None, F.empty_complex(p_even), None)]
    torch.cuda.synchronize()
    F.fft3d_batch_submit(items)
    torch.cuda.synchronize()
    assert bool((items[0][3] == X).all()) and bool((items[0][4] == y_free).all())
    assert bool((items[1][4] == X_even).all())
    with pytest.raises(F.Fft3dError) as e:
        F.Batch(items[:1])
    assert e.value.code == F.FFT3D_ERR_UNSUPPORTED
    with pytest.raises(F.Fft3dError) as e:
        F.r2c_pruned(plan, xd, (5, 5, 5))
    assert e.value.code == F.FFT3D_ERR_UNSUPPORTED
