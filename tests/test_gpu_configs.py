"""Parity at the workload sizes, in the launch configuration the benchmark times.

* 32^3 FP64, uniform[-1,1] (seed 1): full comparison with the oracle, the
  separable naive DFT (the definition, axis by axis) and the round trip.
* 256^3 FP64, k^(-5/3) field with |k| <= 85 (seed 2): full comparison.
* 512^3 FP32 and FP64, k^(-5/3) field (seed 3): full comparison with the
  oracle (all host threads), r2c and c2r.
* 1024^3 FP32 and FP64, the same k^(-5/3) construction (seed 3): full
  comparison with the oracle, r2c and c2r, plus the round trip
  c2r(r2c(x)) = N x and Parseval's identity on the GPU.
"""
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


@pytest.fixture(scope="module")
def field1024():
    say("1024^3 k53 field (generating on the host)")
    return fields.k53_field((1024, 1024, 1024), seed=3)


def _host_mem_gb() -> float:
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                return int(line.split()[1]) / 2**20
    except OSError:
        pass
    return float("nan")


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_1024cubed_k53_full(F, oracle, field1024, dtype):
    """The whole 1024^3 outputs against the oracle, element by element (rel-L2
    over every stored scalar), plus Parseval and the round trip on the GPU.
    Host memory needed: about 45 GB (FP64) / 35 GB (FP32)."""
    import torch
    shape = (1024, 1024, 1024)
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    say("1024^3 %s (host MemTotal %.0f GiB)" % (dtype, _host_mem_gb()))
    x = rounded(field1024, dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    say("1024^3 %s r2c" % dtype)
    X = F.r2c(plan, xd)
    torch.cuda.synchronize()
    # Parseval: sum x^2 = (1/N) sum w(k2) |X|^2
    w = torch.full((n2 // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = 1.0
    w[n2 // 2] = 1.0
    lhs = float(torch.sum(xd.double() ** 2))
    rhs = float(sum(float(torch.sum(w * (X[i].abs().double() ** 2))) for i in range(n0))) / N
    assert abs(lhs - rhs) / lhs <= TOL[dtype]
    Xg = host(X)
    say("1024^3 %s oracle r2c" % dtype)
    Xo = oracle.r2c(x, threads=oracle_threads())
    del x
    err = rel_l2(Xg, Xo)
    say("1024^3 %s r2c rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]
    del Xg
    # round trip of the GPU spectrum, on the GPU
    work = F.empty_complex(plan)
    y = F.c2r(plan, X, work=work)
    num = float(torch.linalg.vector_norm((y.double() - N * xd.double()).ravel()))
    den = float(torch.linalg.vector_norm((N * xd.double()).ravel()))
    assert num / den <= TOL[dtype]
    del X, y, xd
    # c2r of the oracle spectrum (rounded to the dtype) against the oracle
    S = rounded(Xo, dtype)
    del Xo
    say("1024^3 %s c2r" % dtype)
    Sd = dev_cplx(S, dtype)
    y = host(F.c2r(plan, Sd, work=work))
    del Sd, work
    torch.cuda.empty_cache()
    say("1024^3 %s oracle c2r" % dtype)
    yo = oracle.c2r(S, n2, threads=oracle_threads())
    del S
    err = rel_l2(y, yo)
    say("1024^3 %s c2r rel-L2 %.3e" % (dtype, err))
    assert err <= TOL[dtype]
