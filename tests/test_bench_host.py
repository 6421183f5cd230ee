"""CPU tests of the benchmark's host logic: the byte accountings behind its
bandwidth figures (against the values worked out for 512^3 and 1024^3), and
the single-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pair_bytes_alg_and_min():
    # B_alg: each of the two steps reads and writes the array once per direction
    assert bench.pair_bytes_alg((512, 512, 512), 4) == 4_307_550_208
    assert bench.pair_bytes_alg((512, 512, 512), 8) == 8_615_100_416
    assert abs(bench.pair_bytes_alg((1024, 1024, 1024), 4) / 1e9 - 34.41) < 0.01
    assert bench.pair_bytes_min((512, 512, 512), 4) == 2 * (4 * 512 ** 3 + 8 * 512 * 512 * 257)
    # the split path's three sweeps: sN + 5 * 2sM per direction
    assert bench.pair_bytes_swept((512, 512, 512), 4) == 2 * (4 * 512 ** 3 + 5 * 8 * 512 * 512 * 257)


def test_pass_bytes_sum_to_swept_pair():
    shape = (512, 512, 512)
    for elem in (4, 8):
        assert sum(bench.pass_bytes(p, shape, elem) for p in range(6)) == bench.pair_bytes_swept(shape, elem)


def test_pruned_bytes():
    shape = (512, 512, 512)
    # no cut: the pruned accountings are the full ones
    assert bench.pruned_pair_bytes_alg(shape, 4, (-1, -1, -1)) == bench.pair_bytes_alg(shape, 4)
    assert bench.pruned_pair_bytes_swept(shape, 4, (-1, -1, -1)) == bench.pair_bytes_swept(shape, 4)
    # the two-thirds box: 341 x 341 x 171 kept modes
    k = (170, 170, 170)
    fwd = 4 * 512 ** 3 + 8 * (2 * 512 * 512 * 171 + 2 * 512 * 341 * 171 + 341 * 341 * 171)
    assert bench.pruned_pair_bytes_swept(shape, 4, k) == 2 * fwd
    assert abs(bench.pruned_pair_bytes_swept(shape, 4, k) / bench.pair_bytes_swept(shape, 4) - 0.585) < 0.001
    assert abs(bench.pruned_pair_bytes_alg(shape, 4, k) / bench.pair_bytes_alg(shape, 4) - 0.545) < 0.001


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
