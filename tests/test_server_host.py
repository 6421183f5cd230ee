"""CPU tests of the serving layer's host logic: the arena allocator, and the
server itself in its no-device mode (arena as address arithmetic, host-only
plans, a request completes as soon as it is launched) -- admission by budget,
first-come-first-served order, batched versus single launches, validation,
shutdown with requests that never fit."""
import os
import subprocess
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_1406_5597_amd import fft3d
    return fft3d


def test_arena_random_alloc_free(tmp_path):
    exe = str(tmp_path / "arena_sim")
    r = subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(ROOT, "tests", "arena_sim.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    for seed in (1, 2, 3):
        out = subprocess.run([exe, str(seed)], capture_output=True, text=True, timeout=120).stdout.strip()
        assert out == "ok", out


def cplx_bytes(shape, elem):
    n0, n1, n2 = shape
    return n0 * n1 * (n2 // 2 + 1) * 2 * elem


def fake_inputs(k, base=0x100000):
    return [base + 0x10000 * i for i in range(k)]


def make(F, budget, **kw):
    return F.Server(budget, flags=F.FFT3D_SERVER_NO_DEVICE, **kw)


def test_admission_waits_for_budget(F):
    shape = (16, 16, 16)
    need = 3 * cplx_bytes(shape, 4)  # one 3-field r2c request
    with make(F, 2 * need + 1000) as s:
        ids = [s.submit(shape, "f32", F.FFT3D_R2C, fake_inputs(3)) for _ in range(5)]
        assert s.wait(ids[0], 5.0) and s.wait(ids[1], 5.0)
        assert not s.wait(ids[2], 0.2), "admitted beyond the budget"
        st = s.stats()
        assert st["waiting"] == 3 and st["completed"] == 2
        assert st["peak_reserved_bytes"] <= st["budget_bytes"]
        s.release(ids[0])
        assert s.wait(ids[2], 5.0)
        assert not s.wait(ids[3], 0.2)
        for i in ids[1:3]:
            s.release(i)
        for i in ids[3:]:
            assert s.wait(i, 5.0)
            s.release(i)
        st = s.stats()
        assert st["released"] == 5 and st["reserved_bytes"] == 0
        assert st["peak_reserved_bytes"] <= 2 * need


def test_first_come_first_served(F):
    """A large request at the head waits for room; smaller later ones do not
    pass it."""
    small, large = (8, 8, 8), (32, 32, 32)
    budget = 3 * cplx_bytes(large, 4) + 3 * cplx_bytes(small, 4)
    with make(F, budget) as s:
        a = s.submit(large, "f32", F.FFT3D_R2C, fake_inputs(3))
        assert s.wait(a, 5.0)
        b = s.submit(large, "f32", F.FFT3D_R2C, fake_inputs(3))
        c = s.submit(small, "f32", F.FFT3D_R2C, fake_inputs(3))
        assert not s.wait(b, 0.2) and not s.wait(c, 0.2)
        s.release(a)
        assert s.wait(b, 5.0) and s.wait(c, 5.0)
        _, tb = s.result(b, 3)
        _, tc = s.result(c, 3)
        assert tb[1] <= tc[1], "admission out of arrival order"


def test_batched_and_single_launches(F):
    with make(F, 1 << 30, batch_points=4096) as s:
        small = [s.submit((16, 16, 16), "f64", F.FFT3D_C2R, fake_inputs(2)) for _ in range(3)]
        big = s.submit((32, 32, 32), "f32", F.FFT3D_R2C, fake_inputs(1))
        for i in small + [big]:
            assert s.wait(i, 5.0)
        st = s.stats()
        assert st["single_launches"] >= 1 and st["batched_launches"] >= 1
        # c2r reserves a work buffer per field until completion; outputs remain
        outs, t = s.result(small[0], 2)
        assert len(set(outs)) == 2 and t[0] <= t[1] <= t[2] <= t[3]
        assert st["reserved_bytes"] == 3 * 2 * 16 * 16 * 16 * 8 + cplx_bytes((32, 32, 32), 4)


def test_many_batched_items_split_by_limit(F):
    with make(F, 1 << 30, max_batch_items=4) as s:
        ids = [s.submit((8, 8, 8), "f32", F.FFT3D_R2C, fake_inputs(3)) for _ in range(10)]
        for i in ids:
            assert s.wait(i, 5.0)
        assert s.stats()["batched_launches"] >= 3


def test_validation(F):
    with make(F, 1 << 20) as s:
        with pytest.raises(F.Fft3dError) as e:
            s.submit((64, 64, 64), "f32", F.FFT3D_R2C, fake_inputs(3))  # needs more than the budget
        assert e.value.code == F.FFT3D_ERR_BUDGET
        with pytest.raises(F.Fft3dError) as e:
            s.submit((8, 8, 11), "f32", F.FFT3D_R2C, fake_inputs(1))
        assert e.value.code == F.FFT3D_ERR_UNSUPPORTED
        with pytest.raises(F.Fft3dError):
            s.submit((8, 8, 8), "f32", 7, fake_inputs(1))
        with pytest.raises(F.Fft3dError):
            s.submit((8, 8, 8), "f64", F.FFT3D_R2C, [0x100008])  # misaligned for FP64
        with pytest.raises(F.Fft3dError):
            s.submit((8, 8, 8), "f32", F.FFT3D_R2C, [])
        with pytest.raises(F.Fft3dError):
            s.release(12345)
        i = s.submit((8, 8, 8), "f32", F.FFT3D_R2C, fake_inputs(1))
        assert s.wait(i, 5.0)
        s.release(i)
        with pytest.raises(F.Fft3dError):
            s.result(i, 1)
    with pytest.raises(F.Fft3dError):
        F.Server(0, flags=F.FFT3D_SERVER_NO_DEVICE)


def test_shutdown_drops_what_never_fits(F):
    shape = (16, 16, 16)
    s = make(F, 3 * cplx_bytes(shape, 4) + 512)
    a = s.submit(shape, "f32", F.FFT3D_R2C, fake_inputs(3))
    b = s.submit(shape, "f32", F.FFT3D_R2C, fake_inputs(3))
    assert s.wait(a, 5.0)
    assert not s.wait(b, 0.1)
    waiter = {}

    def wait_b():
        try:
            waiter["r"] = s.wait(b, 10.0)
        except F.Fft3dError as e:
            waiter["r"] = e

    t = threading.Thread(target=wait_b)
    t.start()
    s.close()  # b never fits: dropped, its waiter released with an error
    t.join(10)
    assert isinstance(waiter.get("r"), F.Fft3dError)


def test_concurrent_submitters(F):
    with make(F, 1 << 30) as s:
        ids, lock = [], threading.Lock()

        def client(k):
            for j in range(50):
                i = s.submit((8, 8, 8), ("f32", "f64")[(k + j) % 2], (F.FFT3D_R2C, F.FFT3D_C2R)[j % 2],
                             fake_inputs(3))
                with lock:
                    ids.append(i)

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for i in ids:
            assert s.wait(i, 5.0)
            s.release(i)
        st = s.stats()
        assert st["completed"] == 200 and st["reserved_bytes"] == 0
