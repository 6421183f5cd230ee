"""GPU parity at the extents the plan accepts at most (n0, n1 <= 4096,
n2 <= 8192), against the FP64 oracle: whole arrays where the oracle finishes
in seconds, sampled outputs (the oracle's one-value evaluators) and the round
trip over the whole array where it does not."""
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


FULL = [(4096, 2, 2), (2, 4096, 2), (1, 1, 8192), (3, 2, 8192), (2, 64, 8192), (4096, 3, 6)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", FULL, ids=lambda s: "x".join(map(str, s)))
def test_limit_extents_full_oracle(F, oracle, shape, dtype):
    say("limits %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=41), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    assert rel_l2(host(X), oracle.r2c(x)) <= TOL[dtype]
    y = F.c2r(plan, X, work=F.empty_complex(plan))
    assert rel_l2(host(y), x * np.prod(shape)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(4096, 4096, 2), (4096, 2, 8192), (2, 4096, 8192)],
                         ids=lambda s: "x".join(map(str, s)))
def test_limit_extents_sampled(F, oracle, shape, dtype):
    import torch
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    say("limits sampled %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=42), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(43)
    ks = [(0, 0, 0), (n0 - 1, n1 - 1, n2 // 2), (n0 // 2, n1 // 2, 0)] + [
        (int(rng.integers(n0)), int(rng.integers(n1)), int(rng.integers(n2 // 2 + 1))) for _ in range(5)]
    Xs = host(torch.stack([X[k] for k in ks]))
    ref = np.array([oracle.r2c_point(x, k) for k in ks])
    scale = np.sqrt(np.sum(x.astype(np.float64) ** 2))
    assert np.max(np.abs(Xs - ref)) / scale <= (1e-12 if dtype == "f64" else 5e-6)
    y = F.c2r(plan, X, work=F.empty_complex(plan))
    num = float(torch.linalg.vector_norm((y.double() - N * xd.double()).ravel()))
    den = float(torch.linalg.vector_norm((N * xd.double()).ravel()))
    assert num / den <= TOL[dtype]
