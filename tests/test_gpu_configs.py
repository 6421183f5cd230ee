"""Parity at the workload sizes, in the launch configuration the benchmark times.

* 32^3 FP64, uniform[-1,1] (seed 1): full comparison with the oracle, the
  separable naive DFT (the definition, axis by axis) and the round trip.
* 256^3 FP64, k^(-5/3) field with |k| <= 85 (seed 2): full comparison.
* 512^3 FP32 and FP64, k^(-5/3) field (seed 3): full comparison with the
  oracle (all host threads), r2c and c2r.
* 1024^3 FP32 and FP64: outputs sampled one by one from the oracle's
  definition (O(N) per value), plus properties that hold at any size: the
  round trip c2r(r2c(x)) = N x and Parseval's identity.
"""
import numpy as np
import pytest

from paper_1406_5597_amd import fields
from tests.gpu_util import TOL, dev_cplx, dev_real, host, oracle_threads, rel_l2, rounded, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    return fft3d


def test_32cubed_fp64_uniform(F, oracle):
    shape = (32, 32, 32)
    say("32^3 f64")
    x = fields.uniform(shape, seed=1)
    plan = F.Plan(*shape, dtype="f64")
    X = host(F.r2c(plan, dev_real(x, "f64")))
    assert rel_l2(X, oracle.r2c(x)) <= 1e-12
    # separable naive DFT: the definition, one axis at a time (no FFT anywhere)
    def naive(a, axis, n):
        k = np.arange(n)
        W = np.exp(-2j * np.pi * ((np.outer(k, k)) % n) / n)
        return np.moveaxis(np.tensordot(W, np.moveaxis(a, axis, 0), axes=(1, 0)), 0, axis)
    Xn = naive(naive(naive(x.astype(complex), 2, 32)[:, :, :17], 1, 32), 0, 32)
    assert rel_l2(X, Xn) <= 1e-12
    y = host(F.c2r(plan, dev_cplx(X, "f64")))
    assert rel_l2(y, x * 32 ** 3) <= 1e-12


@pytest.mark.timeout(600)
def test_256cubed_fp64_k53(F, oracle):
    shape = (256, 256, 256)
    say("256^3 f64 k53 (generating)")
    x = fields.k53_field(shape, seed=2, kmax=85)
    plan = F.Plan(*shape, dtype="f64")
    say("256^3 f64 r2c")
    X = host(F.r2c(plan, dev_real(x, "f64")))
    Xo = oracle.r2c(x, threads=oracle_threads())
    assert rel_l2(X, Xo) <= 1e-12
    say("256^3 f64 c2r")
    y = host(F.c2r(plan, dev_cplx(Xo, "f64"), work=F.empty_complex(plan)))
    assert rel_l2(y, oracle.c2r(Xo, 256, threads=oracle_threads())) <= 1e-12


@pytest.fixture(scope="module")
def field512():
    return fields.k53_field((512, 512, 512), seed=3)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_512cubed_k53_full(F, oracle, field512, dtype):
    shape = (512, 512, 512)
    x = rounded(field512, dtype)
    plan = F.Plan(*shape, dtype=dtype)
    say("512^3 %s r2c" % dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    Xg = host(X)
    del xd
    Xo = oracle.r2c(x, threads=oracle_threads())
    err = rel_l2(Xg, Xo)
    say("512^3 %s r2c rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]
    del Xg
    S = rounded(Xo, dtype)
    del Xo
    say("512^3 %s c2r" % dtype)
    y = host(F.c2r(plan, dev_cplx(S, dtype), work=F.empty_complex(plan)))
    yo = oracle.c2r(S, 512, threads=oracle_threads())
    err = rel_l2(y, yo)
    say("512^3 %s c2r rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_1024cubed_sampled_and_properties(F, oracle, dtype):
    import torch
    shape = (1024, 1024, 1024)
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    say("1024^3 %s (generating uniform field)" % dtype)
    x = rounded(fields.uniform(shape, seed=3), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    say("1024^3 %s r2c" % dtype)
    X = F.r2c(plan, xd)
    torch.cuda.synchronize()
    ks = [(0, 0, 0), (1, 2, 3), (1023, 511, 512), (512, 512, 0), (700, 3, 257), (5, 1000, 100)]
    Xs = host(torch.stack([X[k] for k in ks]))
    ref = np.array([oracle.r2c_point(x, k) for k in ks])
    scale = np.sqrt(np.sum(x.astype(np.float64) ** 2))  # typical |X| for white noise
    assert np.max(np.abs(Xs - ref)) / scale <= (1e-12 if dtype == "f64" else 5e-6)
    # Parseval: sum x^2 = (1/N) sum w(k2) |X|^2
    w = torch.full((n2 // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = 1.0
    w[n2 // 2] = 1.0
    lhs = float(torch.sum(xd.double() ** 2))
    rhs = float(torch.sum(w * (X.abs().double() ** 2))) / N
    assert abs(lhs - rhs) / lhs <= (1e-12 if dtype == "f64" else 5e-6)
    say("1024^3 %s c2r" % dtype)
    work = F.empty_complex(plan)
    y = F.c2r(plan, X, work=work)
    del work
    js = [(0, 0, 0), (1023, 1023, 1023), (17, 900, 3)]
    ys = host(torch.stack([y[j] for j in js]))
    Xh = host(X)
    yref = np.array([oracle.c2r_point(Xh, n2, j) for j in js])
    del Xh
    assert np.max(np.abs(ys - yref)) / (N * np.sqrt(np.mean(x.astype(np.float64) ** 2))) <= TOL[dtype]
    # round trip over the whole array, on the GPU side
    num = float(torch.linalg.vector_norm((y.double() - N * xd.double()).ravel()))
    den = float(torch.linalg.vector_norm((N * xd.double()).ravel()))
    assert num / den <= TOL[dtype]
