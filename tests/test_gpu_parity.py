"""GPU parity of the HIP path against the FP64 oracle, element by element.

Every case: the seeded input (rounded to the plan's dtype) goes through the C
ABI on the GPU; the oracle transforms exactly the same values in FP64; the
relative L2 error over all stored scalars must be <= 1e-12 (FP64) or <= 5e-6
(FP32).  Index and layout checks are exact.
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


# shapes chosen to cover: fused small/big plane kernels, the split plane path
# (rows + strided n1 pass), ragged column tiles, radix 2/3/4/8/16 stages,
# length-1 and length-2 axes, n0 != n1 != n2.
SHAPES = [
    (1, 1, 2), (2, 3, 4), (3, 4, 6), (1, 8, 16), (8, 1, 8), (4, 6, 2), (12, 9, 24),
    (16, 6, 12), (27, 8, 18), (32, 32, 32), (48, 36, 64), (96, 64, 32), (64, 96, 128),
    (128, 128, 128), (192, 192, 96), (24, 256, 256), (8, 512, 512), (6, 384, 768),
    (3, 1024, 1024), (1024, 2, 2), (729, 4, 6), (2, 2048, 16), (4, 16, 4096),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_r2c_c2r_match_oracle(F, oracle, shape, dtype):
    say("parity %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=101), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    x_before = xd.clone()
    X = F.r2c(plan, xd)
    Xg = host(X)
    Xo = oracle.r2c(x)
    assert rel_l2(Xg, Xo) <= TOL[dtype], rel_l2(Xg, Xo)
    assert bool((xd == x_before).all()), "r2c modified its input"
    # c2r on the oracle's spectrum (rounded to dtype), with and without work
    S = rounded(Xo, dtype)
    Sd = dev_cplx(S, dtype)
    S_before = Sd.clone()
    work = F.empty_complex(plan)
    y = F.c2r(plan, Sd, work=work)
    yo = oracle.c2r(S, shape[2])
    assert rel_l2(host(y), yo) <= TOL[dtype]
    assert bool((Sd == S_before).all()), "c2r with work modified its input"
    y2 = F.c2r(plan, Sd)  # in-place mode: Sd is scratch now
    assert rel_l2(host(y2), yo) <= TOL[dtype]
    # round trip through the GPU both ways: c2r(r2c(x)) = N x
    y3 = F.c2r(plan, X)
    assert rel_l2(host(y3), x * np.prod(shape)) <= TOL[dtype]


# planes larger than LDS: the two-kernel split path (default) and the
# cooperative one-launch plane step share their tile code, so they agree bit
# for bit
# (2 x 2048 x 16 only in FP64: in FP32 its plane fits LDS and is fused)
BIG_PLANES = [(24, 256, 256), (8, 512, 512), (6, 384, 768), (4, 16, 4096), (6, 512, 96), (16, 288, 576),
              (4, 96, 1536)]


@pytest.mark.parametrize("shape,dtype", [(s, d) for s in BIG_PLANES for d in ("f64", "f32")] + [((2, 2048, 16), "f64")],
                         ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else v)
def test_cooperative_plane_step_matches_split_and_oracle(F, oracle, shape, dtype):
    say("coop vs split %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=202), dtype)
    pc = F.Plan(*shape, dtype=dtype, coop_plane=True)
    ps = F.Plan(*shape, dtype=dtype)
    if pc.describe()["plane"]["kind"] != "coop":
        pytest.skip("plane fits LDS in %s" % dtype)
    assert ps.describe()["plane"]["kind"] == "split"
    xd = dev_real(x, dtype)
    Xc = F.r2c(pc, xd)
    Xs = F.r2c(ps, xd)
    assert bool((Xc == Xs).all())
    assert rel_l2(host(Xc), oracle.r2c(x)) <= TOL[dtype]
    for work in (True, False):
        yc = F.c2r(pc, Xc.clone(), work=F.empty_complex(pc) if work else None)
        ys = F.c2r(ps, Xs.clone(), work=F.empty_complex(ps) if work else None)
        assert bool((yc == ys).all())
        assert rel_l2(host(yc), x * np.prod(shape)) <= TOL[dtype]
    # repeated calls on one plan reuse its counter block
    for _ in range(3):
        assert bool((F.r2c(pc, xd) == Xc).all())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2r_non_hermitian_follows_definition(F, oracle, dtype):
    # arbitrary complex half spectrum: Im of the self-conjugate bins of each
    # row is dropped after the n0/n1 passes, exactly as the oracle defines
    shape = (6, 8, 12)
    say("non-hermitian c2r %s" % dtype)
    rng = np.random.default_rng(5)
    h = shape[2] // 2 + 1
    S = rounded(rng.standard_normal((6, 8, h)) + 1j * rng.standard_normal((6, 8, h)), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    y = host(F.c2r(plan, dev_cplx(S, dtype), work=F.empty_complex(plan)))
    assert rel_l2(y, oracle.c2r_direct(S, shape[2])) <= TOL[dtype]
    S2 = S.copy()
    S2[0, 0, 0] += 3j
    S2[0, 0, h - 1] -= 2j
    y2 = host(F.c2r(plan, dev_cplx(S2, dtype), work=F.empty_complex(plan)))
    assert rel_l2(y2, y) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m", [(1, 2, 3), (5, 3, 7), (-2, 7, 1), (3, 0, 0), (0, 5, 8)])
def test_single_mode_index_map_exact(F, m, dtype):
    # cos of one mode: the peak lands at exactly (m0 mod n0, m1 mod n1, m2)
    # in natural order (a transposed or reversed layout would not)
    shape = (12, 16, 16)
    n0, n1, n2 = shape
    say("single mode %s %s" % (m, dtype))
    j0, j1, j2 = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    x = np.cos(2 * np.pi * (m[0] * j0 / n0 + m[1] * j1 / n1 + m[2] * j2 / n2))
    plan = F.Plan(*shape, dtype=dtype)
    X = host(F.r2c(plan, dev_real(x, dtype)))
    N = n0 * n1 * n2
    a = (m[0] % n0, m[1] % n1, m[2])
    b = ((-m[0]) % n0, (-m[1]) % n1, m[2])
    expect = np.zeros(X.shape, complex)
    expect[a] += N / 2
    if m[2] in (0, n2 // 2):
        expect[b] += N / 2
    big = np.abs(expect) > 0
    assert set(zip(*np.nonzero(np.abs(X) > N * 1e-3))) == set(zip(*np.nonzero(big)))
    assert np.max(np.abs(X - expect)) < N * (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_delta_and_constant(F, dtype):
    shape = (24, 18, 32)
    n0, n1, n2 = shape
    say("delta/constant %s" % dtype)
    plan = F.Plan(*shape, dtype=dtype)
    x = np.zeros(shape)
    a = (5, 11, 7)
    x[a] = 1.0
    X = host(F.r2c(plan, dev_real(x, dtype)))
    k0, k1, k2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2 // 2 + 1), indexing="ij")
    N = n0 * n1 * n2
    e = (k0 * a[0] * n1 * n2 + k1 * a[1] * n0 * n2 + k2 * a[2] * n0 * n1) % N
    assert np.max(np.abs(X - np.exp(-2j * np.pi * e / N))) < (1e-14 if dtype == "f64" else 2e-6)
    Xc = host(F.r2c(plan, dev_real(np.full(shape, 0.5), dtype)))
    expect = np.zeros_like(Xc)
    expect[0, 0, 0] = 0.5 * N
    assert np.max(np.abs(Xc - expect)) < N * (1e-15 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("shape,dtype", [((64, 48, 96), "f64"), ((8, 512, 512), "f32"), ((16, 96, 192), "f32")])
def test_deterministic(F, shape, dtype):
    say("determinism %s %s" % (shape, dtype))
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(fields.uniform(shape, seed=7), dtype)
    X0 = F.r2c(plan, xd)
    y0 = F.c2r(plan, X0, work=F.empty_complex(plan))
    for _ in range(5):
        X = F.r2c(plan, xd)
        assert bool((X == X0).all())
        y = F.c2r(plan, X, work=F.empty_complex(plan))
        assert bool((y == y0).all())


def test_error_paths_on_device(F):
    import torch
    say("error paths")
    plan = F.Plan(8, 8, 8, "f32")
    x = torch.zeros(8 * 8 * 8 + 16, dtype=torch.float32, device="cuda")
    X = torch.zeros(8 * 8 * 5 + 8, dtype=torch.complex64, device="cuda")
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_r2c(plan, x.data_ptr() + 4, X)
    assert e.value.code == F.FFT3D_ERR_ALIGN
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_r2c(plan, x, x.data_ptr() + 64)
    assert e.value.code == F.FFT3D_ERR_INVALID_ARG
    with pytest.raises(F.Fft3dError) as e:
        F.fft3d_c2r(plan, X, x, work=X.data_ptr() + 64)
    assert e.value.code == F.FFT3D_ERR_INVALID_ARG
    with pytest.raises(F.Fft3dError):
        F.fft3d_r2c(plan, 0, X)
    torch.cuda.synchronize()


def test_batch_submit_matches_alone(F):
    import torch
    shapes = [((32, 32, 32), "f64"), ((48, 48, 48), "f32"), ((64, 64, 64), "f64"), ((96, 96, 96), "f32"),
              ((128, 128, 128), "f32"), ((192, 192, 96), "f64")]
    say("batch_submit mixed")
    items, alone, outs = [], [], []
    plans = []
    for i, (s, d) in enumerate(shapes):
        p = F.Plan(*s, dtype=d)
        plans.append(p)
        x = dev_real(fields.uniform(s, seed=1000 + i), d)
        X1 = F.r2c(p, x)
        y1 = F.c2r(p, X1.clone(), work=F.empty_complex(p))
        alone.append((X1, y1))
        mid, y = F.empty_complex(p), F.empty_real(p)
        outs.append((mid, y))
        items.append((p, F.FFT3D_ROUNDTRIP, x, mid, y, F.empty_complex(p)))
    F.fft3d_batch_submit(items)
    torch.cuda.synchronize()
    for (X1, y1), (mid, y) in zip(alone, outs):
        assert bool((mid == X1).all())
        assert bool((y == y1).all())


TRANSPOSED_SHAPES = [(2, 3, 4), (1, 8, 16), (8, 1, 8), (12, 9, 24), (32, 32, 32), (48, 36, 64), (96, 64, 32),
                     (24, 256, 256), (128, 128, 128), (3, 1024, 1024), (1024, 4, 36)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", TRANSPOSED_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_transpose_based_method(F, oracle, shape, dtype):
    """The paper's transpose-based method (plane step, explicit n0<->n1
    exchange, contiguous-in-slab n0 columns) gives the transpose of the
    transpose-free spectrum bit for bit, and its inverse the same real field."""
    import torch
    say("transposed %s %s" % (shape, dtype))
    n0, n1, n2 = shape
    x = rounded(fields.uniform(shape, seed=77), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    Xt = torch.empty((n1, n0, n2 // 2 + 1), dtype=X.dtype, device="cuda")
    work = F.empty_complex(plan)
    F.fft3d_r2c_transposed(plan, xd, Xt, work)
    torch.cuda.synchronize()
    assert bool((Xt == X.permute(1, 0, 2)).all()), "transposed spectrum differs from the transpose-free one"
    assert rel_l2(host(Xt).transpose(1, 0, 2), oracle.r2c(x)) <= TOL[dtype]
    y_free = F.c2r(plan, X.clone(), work=F.empty_complex(plan))
    y = F.empty_real(plan)
    F.fft3d_c2r_transposed(plan, Xt, y, work)
    torch.cuda.synchronize()
    assert bool((y == y_free).all()), "transposed inverse differs"


def test_transposed_needs_work(F):
    p = F.Plan(8, 8, 8, dtype="f32")
    x = dev_real(fields.uniform((8, 8, 8), 1), "f32")
    Xt = F.empty_complex(p)
    with pytest.raises(F.Fft3dError):
        F.fft3d_r2c_transposed(p, x, Xt, None)
    with pytest.raises(F.Fft3dError):
        F.fft3d_c2r_transposed(p, Xt, F.empty_real(p), None)
