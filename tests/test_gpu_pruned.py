"""GPU tests of the pruned (dealiased) transforms.

fft3d_r2c_pruned must equal fft3d_r2c bit for bit on the kept box and leave
the bins k2 > K2 untouched (the rows, columns and planes outside the box are
never written there); fft3d_c2r_pruned must equal fft3d_c2r of the spectrum
zeroed outside the box value for value while never reading outside the box
(NaN planted there must not reach the output).  Both are also checked against
the oracle's pruned transforms, within the parity bounds."""
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
    return fft3d


def third(shape):
    """The two-thirds rule: |k| <= n/3 on every axis."""
    return tuple(n // 3 for n in shape)


# fused planes, split planes (rows kernel + n1 pass), length-1 axes, ragged
# column tiles (K2 + 1 not a multiple of the tile width), 3-smooth lengths
SHAPES = [(2, 3, 4), (8, 1, 8), (1, 8, 16), (12, 9, 24), (32, 32, 32), (48, 36, 64), (96, 64, 32),
          (24, 256, 256), (128, 128, 128), (8, 512, 512), (6, 384, 768), (3, 1024, 1024)]


def box_host(shape, kmax):
    import oracle
    return oracle.box_mask(shape, kmax)


def check_pair(F, oracle, shape, dtype, kmax, coop=False, seed=61):
    import torch
    n0, n1, n2 = shape
    plan = F.Plan(*shape, dtype=dtype, coop_plane=coop)
    x = rounded(fields.uniform(shape, seed=seed), dtype)
    xd = dev_real(x, dtype)
    mask = box_host(shape, kmax)
    mask_d = torch.from_numpy(mask).to("cuda")
    # forward: kept box bit for bit, bins beyond K2 untouched
    Xf = F.r2c(plan, xd)
    Xp = F.empty_complex(plan)
    Xp.fill_(complex(float("nan"), float("nan")))
    F.r2c_pruned(plan, xd, kmax, X=Xp)
    torch.cuda.synchronize()
    assert bool((Xp[mask_d] == Xf[mask_d]).all()), "pruned r2c differs from r2c on the kept box"
    K2 = kmax[2]
    if 0 <= K2 < n2 // 2:
        assert bool(torch.isnan(Xp[:, :, K2 + 1:].real).all()), "pruned r2c wrote beyond K2"
    Xo = oracle.r2c_pruned(x, kmax)
    assert rel_l2(host(Xp)[mask], Xo[mask]) <= TOL[dtype]
    # inverse: NaN outside the box must not be read
    Xz = Xf.clone()
    Xz[~mask_d] = 0
    y_full = F.c2r(plan, Xz.clone(), work=F.empty_complex(plan))
    Xn = Xf.clone()
    Xn[~mask_d] = complex(float("nan"), float("nan"))
    Xn_before = Xn.clone()
    yp = F.c2r_pruned(plan, Xn, kmax, work=F.empty_complex(plan))
    torch.cuda.synchronize()
    assert bool((yp == y_full).all()), "pruned c2r differs from c2r of the zeroed spectrum"
    assert bool(((Xn == Xn_before) | (torch.isnan(Xn.real) & torch.isnan(Xn_before.real))).all()), \
        "pruned c2r with work modified X"
    yp2 = F.c2r_pruned(plan, Xn.clone(), kmax)  # in place: X is scratch
    assert bool((yp2 == y_full).all()), "pruned c2r without work differs"
    yo = oracle.c2r_pruned(host(Xf).astype(np.complex128), n2, kmax)
    assert rel_l2(host(yp), yo) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_pruned_two_thirds(F, oracle, shape, dtype):
    say("pruned 2/3 %s %s" % (shape, dtype))
    check_pair(F, oracle, shape, dtype, third(shape))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,kmax", [((32, 32, 32), (-1, -1, -1)), ((48, 36, 64), (0, 0, 0)),
                                        ((48, 36, 64), (23, 17, 32)), ((96, 64, 32), (-1, 5, 3)),
                                        ((24, 256, 256), (3, -1, 100)), ((128, 128, 128), (63, 63, 64)),
                                        ((12, 9, 24), (5, 4, 11))],
                         ids=lambda v: "x".join(map(str, v)))
def test_pruned_other_boxes(F, oracle, shape, kmax, dtype):
    """Whole axes, single modes, boxes one short of the full axis (the
    Nyquist row dropped), and asymmetric cuts."""
    say("pruned box %s %s %s" % (shape, kmax, dtype))
    check_pair(F, oracle, shape, dtype, kmax)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pruned_on_cooperative_plan(F, oracle, dtype):
    """A plan whose full transform runs the cooperative plane step: the pruned
    path takes the split kernels, which agree with it bit for bit."""
    shape = (8, 512, 512)
    say("pruned coop plan %s %s" % (shape, dtype))
    p = F.Plan(*shape, dtype=dtype, coop_plane=True)
    if p.describe()["plane"]["kind"] != "coop":
        pytest.skip("plane fits LDS")
    check_pair(F, oracle, shape, dtype, third(shape), coop=True)


def test_pruned_unbounded_box_is_the_full_transform(F):
    import torch
    shape = (32, 48, 64)
    say("pruned full box %s" % (shape,))
    plan = F.Plan(*shape, dtype="f64")
    xd = dev_real(fields.uniform(shape, 3), "f64")
    X = F.r2c(plan, xd)
    for kmax in ((-1, -1, -1), (16, 24, 32), (100, 100, 100)):
        Xp = F.r2c_pruned(plan, xd, kmax)
        assert bool((Xp == X).all())
        y = F.c2r(plan, X.clone(), work=F.empty_complex(plan))
        yp = F.c2r_pruned(plan, X.clone(), kmax, work=F.empty_complex(plan))
        assert bool((yp == y).all())
    torch.cuda.synchronize()


def test_pruned_errors(F):
    plan = F.Plan(16, 16, 16, dtype="f32")
    x = dev_real(fields.uniform((16, 16, 16), 1), "f32")
    X = F.empty_complex(plan)
    with pytest.raises(F.Fft3dError):
        F.fft3d_r2c_pruned(plan, x, X, None)
    with pytest.raises(F.Fft3dError):
        F.fft3d_c2r_pruned(plan, X, F.empty_real(plan), None)
    with pytest.raises(F.Fft3dError):  # X overlapping x
        F.fft3d_r2c_pruned(plan, x, x, (5, 5, 5))
    with pytest.raises(ValueError):
        F.fft3d_r2c_pruned(plan, x, X, (5, 5))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_pruned_512cubed_bench_configuration(F, oracle, dtype):
    """The benchmark's pruned pair (512^3, K = 170 on every axis): bit for bit
    against the full transforms on the whole box, and sampled kept modes
    against the oracle's one-value evaluator."""
    import torch
    shape = (512, 512, 512)
    kmax = (170, 170, 170)
    say("pruned 512^3 %s" % dtype)
    plan = F.Plan(*shape, dtype=dtype)
    x = rounded(fields.uniform(shape, seed=71), dtype)
    xd = dev_real(x, dtype)
    Xf = F.r2c(plan, xd)
    Xp = F.r2c_pruned(plan, xd, kmax)
    mask = torch.from_numpy(oracle.box_mask(shape, kmax)).to("cuda")
    assert bool((Xp[mask] == Xf[mask]).all())
    for k in [(0, 0, 0), (170, 342, 170), (342, 170, 1), (5, 500, 99)]:
        want = oracle.r2c_point(x, k)
        got = complex(Xp[k].item())
        scale = np.sqrt(np.sum(x.astype(np.float64) ** 2))
        assert abs(got - want) / scale <= (1e-12 if dtype == "f64" else 5e-6), (k, got, want)
    Xf[~mask] = 0
    y_full = F.c2r(plan, Xf, work=F.empty_complex(plan))
    del Xf
    yp = F.c2r_pruned(plan, Xp, kmax, work=F.empty_complex(plan))
    torch.cuda.synchronize()
    assert bool((yp == y_full).all())
