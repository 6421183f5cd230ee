"""GPU tests of the served form: requests of 3-component fields arriving
while others run, admitted under a small HBM budget so that some must wait,
launched in batches (small shapes) or alone (larger ones) on several streams.
Each result must be bit-identical to the same transform run alone through
fft3d_r2c / fft3d_c2r (which the parity tests pin to the FP64 oracle); a few
are also checked against the oracle here."""
import threading
import time

import numpy as np
import pytest

from workloads import fields
from tests.gpu_util import TOL, dev_cplx, dev_real, host, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_5597_amd import fft3d
    return fft3d


SHAPES = [(32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 128, 128), (64, 64, 32)]


class Pool:
    """Per (shape, dtype): three real components and three spectra on the
    device, from the numpy generators (seeded), and the plan."""

    def __init__(self, F, shape, dtype, seed):
        self.plan = F.Plan(*shape, dtype=dtype)
        u = fields.velocity_field(shape, seed)
        U = fields.velocity_spectrum(shape, seed + 1)
        self.real = [dev_real(fields.as_dtype(u[c], dtype), dtype) for c in range(3)]
        self.spec = [dev_cplx(fields.as_dtype(U[c], dtype), dtype) for c in range(3)]


def alone(F, pool, direction):
    """The same transform through the single-item entry points."""
    import torch
    p = pool.plan
    if direction == F.FFT3D_R2C:
        out = [F.r2c(p, x) for x in pool.real]
    else:
        out = [F.c2r(p, X.clone(), work=F.empty_complex(p)) for X in pool.spec]
    torch.cuda.synchronize()
    return out


def test_served_requests_match_alone(F, oracle):
    import torch
    say("server: mixed stream")
    rng = np.random.default_rng(21)
    pools = {}
    for i, s in enumerate(SHAPES):
        for d in ("f32", "f64"):
            pools[(s, d)] = Pool(F, s, d, 3000 + 10 * i + (d == "f64"))
    ref = {(k, r): alone(F, pools[k], r) for k in pools for r in (F.FFT3D_R2C, F.FFT3D_C2R)}
    # budget: the largest request (128^3 FP64 c2r: 3 outputs + 3 work) and a bit
    budget = 3 * (128 ** 3 * 8 + 128 * 128 * 65 * 16) + (8 << 20)
    n = 80
    reqs = [(SHAPES[int(rng.integers(len(SHAPES)))], ("f32", "f64")[int(rng.random() < 0.3)], int(rng.integers(2)))
            for _ in range(n)]
    gaps = rng.exponential(1.0 / 400.0, size=n)
    results, errors = {}, []
    with F.Server(budget, nstreams=3, batch_points=100000) as srv:
        ids = [None] * n

        def producer():
            for i, (s, d, r) in enumerate(reqs):
                time.sleep(gaps[i])
                p = pools[(s, d)]
                ids[i] = srv.submit(s, d, r, p.real if r == F.FFT3D_R2C else p.spec)

        def consumer():
            try:
                for i in range(n):
                    while ids[i] is None:
                        time.sleep(1e-4)
                    assert srv.wait(ids[i], 60.0)
                    s, d, r = reqs[i]
                    p = pools[(s, d)]
                    outs, t = srv.result(ids[i], 3)
                    like = ref[((s, d), r)]
                    got = []
                    for c in range(3):
                        dst = torch.empty_like(like[c])
                        F.copy_from_device(dst, outs[c], dst.numel() * dst.element_size())
                        got.append(dst)
                    results[i] = (got, t)
                    srv.release(ids[i])
            except Exception as e:  # reported in the main thread
                errors.append(e)

        tp = threading.Thread(target=producer)
        tc = threading.Thread(target=consumer)
        tp.start()
        tc.start()
        tp.join()
        tc.join(120)
        assert not errors, errors
        st = srv.stats()
    assert st["completed"] == n and st["released"] == n and st["reserved_bytes"] == 0
    assert st["peak_reserved_bytes"] <= budget
    assert st["batched_launches"] > 0 and st["single_launches"] > 0
    for i, (s, d, r) in enumerate(reqs):
        got, t = results[i]
        like = ref[((s, d), r)]
        for c in range(3):
            assert bool((got[c] == like[c]).all()), "request %d (%s %s dir %d) component %d differs" % (i, s, d, r, c)
        assert t[0] <= t[1] <= t[2] <= t[3]
    # inputs untouched by the c2r requests (work buffers keep them intact)
    for (s, d), p in pools.items():
        U = fields.velocity_spectrum(s, 3000 + 10 * SHAPES.index(s) + (d == "f64") + 1)
        assert np.array_equal(host(p.spec[0]), fields.as_dtype(U[0], d))
    # a few against the oracle
    for key in [((32, 32, 32), "f64"), ((64, 64, 32), "f32")]:
        p = pools[key]
        x = host(p.real[1]).astype(np.float64)
        e = rel_l2(host(ref[(key, F.FFT3D_R2C)][1]), oracle.r2c(x))
        assert e <= TOL[key[1]], (key, e)


def test_server_budget_error_and_reuse(F):
    say("server: budget and reuse")
    p = F.Plan(32, 32, 32, dtype="f32")
    x = dev_real(fields.uniform((32, 32, 32), 5), "f32")
    with F.Server(1 << 20) as srv:
        with pytest.raises(F.Fft3dError) as e:
            srv.submit((64, 64, 64), "f32", F.FFT3D_R2C, [x, x, x])
        assert e.value.code == F.FFT3D_ERR_BUDGET
        want = F.r2c(p, x)
        for _ in range(5):  # the arena block is reused request after request
            i = srv.submit((32, 32, 32), "f32", F.FFT3D_R2C, [x])
            assert srv.wait(i, 30.0)
            outs, _ = srv.result(i, 1)
            import torch
            got = torch.empty_like(want)
            F.copy_from_device(got, outs[0], got.numel() * got.element_size())
            assert bool((got == want).all())
            srv.release(i)


def test_server_radix57_and_odd_n2_requests(F):
    """Requests whose plans the batched kernel does not take (radix-5/7
    extents, odd n2) are served through the batch submit's own-kernel path:
    bit for bit the transforms run alone."""
    import torch
    say("server: radix-5/7 and odd n2")
    shapes = [((35, 45, 28), "f32"), ((16, 16, 15), "f64"), ((32, 32, 32), "f32")]
    with F.Server(1 << 30, nstreams=2, batch_points=1 << 20) as srv:
        for i, (s, d) in enumerate(shapes):
            p = F.Plan(*s, dtype=d)
            xs = [dev_real(fields.as_dtype(fields.uniform(s, 600 + 3 * i + c), d), d) for c in range(3)]
            want = [F.r2c(p, x) for x in xs]
            torch.cuda.synchronize()
            rid = srv.submit(s, d, F.FFT3D_R2C, xs)
            assert srv.wait(rid, 30.0)
            outs, _ = srv.result(rid, 3)
            for c in range(3):
                got = torch.empty_like(want[c])
                F.copy_from_device(got, outs[c], got.numel() * got.element_size())
                assert bool((got == want[c]).all()), (s, d, c)
            srv.release(rid)
        st = srv.stats()
    assert st["batched_launches"] >= 1


def test_server_large_requests(F, oracle):
    """Requests at the sizes of the served workload's large end (256^3 and
    512^3 FP32, 256x256x128 FP64; forward and inverse), served alone under
    the budget: bit for bit the transforms run alone, and sampled outputs of
    the 512^3 request against the oracle's point evaluator."""
    import torch
    say("server: large requests")
    specs = [((256, 256, 256), "f32", F.FFT3D_R2C, 3), ((256, 256, 256), "f32", F.FFT3D_C2R, 3),
             ((256, 256, 128), "f64", F.FFT3D_C2R, 2), ((512, 512, 512), "f32", F.FFT3D_R2C, 1)]
    with F.Server(6 << 30, nstreams=2, batch_points=1 << 20) as srv:
        for i, (s, d, r, nc) in enumerate(specs):
            p = F.Plan(*s, dtype=d)
            xs = [dev_real(fields.as_dtype(fields.uniform(s, 700 + 5 * i + c), d), d) for c in range(nc)]
            if r == F.FFT3D_R2C:
                ins = xs
                want = [F.r2c(p, x) for x in xs]
            else:
                ins = [F.r2c(p, x) for x in xs]
                want = [F.c2r(p, X.clone(), work=F.empty_complex(p)) for X in ins]
            torch.cuda.synchronize()
            rid = srv.submit(s, d, r, ins)
            assert srv.wait(rid, 60.0)
            outs, _ = srv.result(rid, nc)
            for c in range(nc):
                got = torch.empty_like(want[c])
                F.copy_from_device(got, outs[c], got.numel() * got.element_size())
                assert bool((got == want[c]).all()), (s, d, r, c)
            if s == (512, 512, 512):
                x = host(xs[0]).astype(np.float64)
                Xg = host(got)
                scale = np.sqrt(np.sum(x * x))  # the same bound as the sampled parity tests
                for k in [(0, 0, 0), (3, 511, 17), (256, 100, 256), (511, 1, 1)]:
                    ref = oracle.r2c_point(x, k)
                    assert abs(Xg[k] - ref) / scale <= 5e-6, (k, Xg[k], ref)
            srv.release(rid)
            del xs, ins, want
        st = srv.stats()
    assert st["completed"] == len(specs) and st["reserved_bytes"] == 0
