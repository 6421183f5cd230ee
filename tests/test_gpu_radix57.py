"""GPU parity for extents with prime factors 5 and 7 (radix-5 and radix-7
stages), against the FP64 oracle: fused and split plane steps, long columns,
mixed 2/3/5/7 schedules; and the other entry points (pruned, transposed,
batched) on such shapes, bit for bit against the plain transforms."""
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


SHAPES = [(5, 7, 10), (25, 49, 70), (125, 14, 20), (35, 45, 28), (343, 6, 14), (60, 210, 210),
          (20, 500, 500), (14, 980, 196), (2401, 2, 2), (6, 700, 1400), (7, 5, 4096)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_radix57_match_oracle(F, oracle, shape, dtype):
    say("radix57 parity %s %s" % (shape, dtype))
    x = rounded(fields.uniform(shape, seed=57), dtype)
    plan = F.Plan(*shape, dtype=dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    Xo = oracle.r2c(x)
    assert rel_l2(host(X), Xo) <= TOL[dtype], rel_l2(host(X), Xo)
    S = rounded(Xo, dtype)
    Sd = dev_cplx(S, dtype)
    y = F.c2r(plan, Sd, work=F.empty_complex(plan))
    yo = oracle.c2r(S, shape[2])
    assert rel_l2(host(y), yo) <= TOL[dtype]
    y2 = F.c2r(plan, Sd)  # in place
    assert rel_l2(host(y2), yo) <= TOL[dtype]
    y3 = F.c2r(plan, X)
    assert rel_l2(host(y3), x * np.prod(shape)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_radix57_single_modes_exact_index(F, dtype):
    """A single cosine mode per axis lands on exactly its two bins."""
    import torch
    shape = (35, 25, 14)
    n0, n1, n2 = shape
    say("radix57 single modes %s" % dtype)
    plan = F.Plan(*shape, dtype=dtype)
    j0, j1, j2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    for m in [(1, 0, 0), (0, 3, 0), (0, 0, 5), (17, 12, 6), (34, 24, 1)]:
        x = np.cos(2 * np.pi * (m[0] * j0 / n0 + m[1] * j1 / n1 + m[2] * j2 / n2))
        X = host(F.r2c(plan, dev_real(rounded(x, dtype), dtype)))
        torch.cuda.synchronize()
        big = np.argwhere(np.abs(X) > 0.25 * x.size)
        want = {(m[0] % n0, m[1] % n1, m[2])}
        if m[2] == 0:
            want.add(((-m[0]) % n0, (-m[1]) % n1, 0))
        assert {tuple(v) for v in big} == want, (m, big)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_radix57_other_entry_points(F, oracle, dtype):
    import torch
    shape = (60, 210, 210)
    n0, n1, n2 = shape
    say("radix57 pruned/transposed %s" % dtype)
    plan = F.Plan(*shape, dtype=dtype)
    x = rounded(fields.uniform(shape, seed=58), dtype)
    xd = dev_real(x, dtype)
    X = F.r2c(plan, xd)
    # pruned, two-thirds box
    kmax = (n0 // 3, n1 // 3, n2 // 3)
    mask = torch.from_numpy(oracle.box_mask(shape, kmax)).to("cuda")
    Xp = F.r2c_pruned(plan, xd, kmax)
    assert bool((Xp[mask] == X[mask]).all())
    Xz = X.clone()
    Xz[~mask] = 0
    y_full = F.c2r(plan, Xz.clone(), work=F.empty_complex(plan))
    yp = F.c2r_pruned(plan, X.clone(), kmax, work=F.empty_complex(plan))
    assert bool((yp == y_full).all())
    # transpose-based method
    Xt = torch.empty((n1, n0, n2 // 2 + 1), dtype=X.dtype, device="cuda")
    work = F.empty_complex(plan)
    F.fft3d_r2c_transposed(plan, xd, Xt, work)
    torch.cuda.synchronize()
    assert bool((Xt == X.permute(1, 0, 2)).all())


def test_radix57_batch_matches_alone(F):
    import torch
    say("radix57 batch")
    shapes = [((35, 45, 28), "f32"), ((25, 49, 70), "f64"), ((60, 210, 210), "f32"), ((5, 7, 10), "f64"),
              ((125, 14, 20), "f32")]
    items, want = [], []
    for i, (s, d) in enumerate(shapes):
        p = F.Plan(*s, dtype=d)
        x = dev_real(fields.uniform(s, 900 + i), d)
        X = F.r2c(p, x)
        y = F.c2r(p, X.clone(), work=F.empty_complex(p))
        want.append((X, y))
        items.append((p, F.FFT3D_ROUNDTRIP, x, F.empty_complex(p), F.empty_real(p), F.empty_complex(p)))
    torch.cuda.synchronize()
    F.fft3d_batch_submit(items)
    torch.cuda.synchronize()
    for (p, _, x, mid, out, work), (X, y) in zip(items, want):
        assert bool((mid == X).all()) and bool((out == y).all())


def test_radix57_batch_handle_refused_and_plan_flags(F):
    say("radix57 batch handle")
    p = F.Plan(35, 45, 28, dtype="f32", coop_plane=True)
    d = p.describe()
    assert d["radix57"] is True and d["plane"]["kind"] != "coop"
    assert F.Plan(32, 48, 64, dtype="f32").describe()["radix57"] is False
    x = dev_real(fields.uniform((35, 45, 28), 1), "f32")
    with pytest.raises(F.Fft3dError) as e:
        F.Batch([(p, F.FFT3D_R2C, x, None, F.empty_complex(p), None)])
    assert e.value.code == F.FFT3D_ERR_UNSUPPORTED
