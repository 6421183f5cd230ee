"""GPU tests of arrays of more than 2^31 elements (real and complex): every
index of the path must be 64-bit safe.

The input is a sum of two separable terms, x = a(j0) b(j1) c(j2) +
d(j0) e(j1) f(j2), with seeded uniform[-1, 1] vectors.  By separability of
the DFT its half spectrum is X = A B C + D E F (outer products of the 1D DFTs
of the vectors), and the oracle's 1D FFT gives those in FP64.  So the whole
output, every one of its more than 2^31 bins, is compared element by element
(relative L2, computed on the GPU plane group by plane group), and c2r of
the GPU spectrum against N x, element by element as well."""
import numpy as np
import pytest

from tests.gpu_util import TOL, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    return fft3d


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_arrays_beyond_2_31_elements(F, oracle, dtype):
    import torch
    shape = (2048, 2048, 1024)
    n0, n1, n2 = shape
    h = n2 // 2 + 1
    N = n0 * n1 * n2
    assert N > 2 ** 31 and n0 * n1 * h > 2 ** 31
    rng = np.random.default_rng(91)
    vecs = [rng.uniform(-1.0, 1.0, size=n) for n in (n0, n1, n2, n0, n1, n2)]
    dev = [torch.from_numpy(v).to("cuda") for v in vecs]
    rdt, cdt = F.torch_dtypes(dtype)
    say("beyond 2^31 %s: input" % dtype)
    x = torch.empty(shape, dtype=rdt, device="cuda")
    G = 64  # planes per group of the on-device arithmetic
    for a0 in range(0, n0, G):
        b0 = min(n0, a0 + G)
        t = (dev[0][a0:b0, None, None] * dev[1][None, :, None] * dev[2][None, None, :] +
             dev[3][a0:b0, None, None] * dev[4][None, :, None] * dev[5][None, None, :])
        x[a0:b0] = t.to(rdt)
        del t
    plan = F.Plan(*shape, dtype=dtype)
    say("beyond 2^31 %s: r2c" % dtype)
    X = F.r2c(plan, x)
    torch.cuda.synchronize()
    # the expected half spectrum from the oracle's 1D FFTs
    S = [torch.from_numpy(oracle.fft1d(v)).to("cuda") for v in vecs]
    S[2], S[5] = S[2][:h], S[5][:h]
    num = den = 0.0
    for a0 in range(0, n0, G):
        b0 = min(n0, a0 + G)
        E = (S[0][a0:b0, None, None] * S[1][None, :, None] * S[2][None, None, :] +
             S[3][a0:b0, None, None] * S[4][None, :, None] * S[5][None, None, :])
        num += float(torch.linalg.vector_norm((X[a0:b0].to(torch.complex128) - E).ravel())) ** 2
        den += float(torch.linalg.vector_norm(E.ravel())) ** 2
        del E
    err = (num / den) ** 0.5
    say("beyond 2^31 %s: r2c rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]
    # c2r of the GPU spectrum (in place, no work buffer) against N x
    say("beyond 2^31 %s: c2r" % dtype)
    y = F.c2r(plan, X)
    torch.cuda.synchronize()
    del X
    num = den = 0.0
    for a0 in range(0, n0, G):
        b0 = min(n0, a0 + G)
        ref = float(N) * x[a0:b0].double()
        num += float(torch.linalg.vector_norm((y[a0:b0].double() - ref).ravel())) ** 2
        den += float(torch.linalg.vector_norm(ref.ravel())) ** 2
        del ref
    err = (num / den) ** 0.5
    say("beyond 2^31 %s: round trip rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]
