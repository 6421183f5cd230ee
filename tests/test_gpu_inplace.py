"""GPU tests of the in-place transforms in FFTW's padded layout: rows of
2*(n2/2+1) reals (n2 used) transformed into the complex spectrum in the same
bytes and back.  Results must be bit for bit those of fft3d_r2c and of
fft3d_c2r without work (same kernels), with NaN in the padding never read;
one case per dtype is also checked against the oracle."""
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


# fused planes, split planes, odd n2, radix 5/7, length-1 axes
SHAPES = [(2, 3, 4), (8, 1, 8), (1, 8, 16), (32, 32, 32), (48, 36, 64), (24, 256, 256), (8, 512, 512),
          (4, 6, 9), (3, 5, 7), (16, 128, 243), (25, 49, 70), (3, 1, 1), (2, 2, 6561)]


def padded(F, plan, x_dev):
    """A padded real buffer holding x (NaN in the padding), and its views."""
    import torch
    n0, n1, n2 = plan.shape
    H = n2 // 2 + 1
    rd, cd = F.torch_dtypes(plan.dtype)
    buf = torch.full((n0, n1, 2 * H), float("nan"), dtype=rd, device="cuda")
    buf[:, :, :n2] = x_dev
    return buf, buf.view(cd)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_inplace_matches_out_of_place(F, oracle, shape, dtype):
    import torch
    say("in place %s %s" % (shape, dtype))
    n0, n1, n2 = shape
    for coop in (False, True):
        plan = F.Plan(*shape, dtype=dtype, coop_plane=coop)
        x = rounded(fields.uniform(shape, seed=31), dtype)
        xd = dev_real(x, dtype)
        X = F.r2c(plan, xd)
        buf, Xv = padded(F, plan, xd)
        F.fft3d_r2c_inplace(plan, buf)
        torch.cuda.synchronize()
        assert Xv.shape == X.shape
        assert bool((Xv == X).all()), "in-place r2c differs"
        y = F.c2r(plan, X.clone())  # no work: the same in-place passes
        F.fft3d_c2r_inplace(plan, Xv)
        torch.cuda.synchronize()
        assert bool((buf[:, :, :n2] == y).all()), "in-place c2r differs"
        if not coop and shape in ((32, 32, 32), (16, 128, 243)):
            assert rel_l2(host(X), oracle.r2c(x)) <= TOL[dtype]
            assert rel_l2(host(buf[:, :, :n2]), x * np.prod(shape)) <= TOL[dtype]


def test_inplace_errors(F):
    p = F.Plan(8, 8, 8, dtype="f64")
    with pytest.raises(F.Fft3dError):
        F.fft3d_r2c_inplace(p, None)
    with pytest.raises(F.Fft3dError):
        F.fft3d_c2r_inplace(p, 0x1008)  # misaligned for complex double
