"""CPU tests of the batched launch's host side: the task lists that
build_batch_table produces, and the ticket protocol the batched kernel runs,
exercised by tests/batch_sim.cpp (the library's own host code, fake device
addresses, the scheduling loop on host threads)."""
import os
import subprocess

import numpy as np
import pytest

from workloads import fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sim") / "batch_sim")
    csrc = os.path.join(ROOT, "paper_1406_5597_amd", "csrc")
    cmd = ["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "batch_sim.cpp"), os.path.join(csrc, "fft3d_plan.cpp"),
           os.path.join(csrc, "fft3d_batch_host.cpp"), "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
           "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("batch_sim build failed:\n" + r.stderr[-3000:])

    def run(lines, workgroups=64, lag=None, mode=None, xcds=None):
        head = ""
        if lag is not None:
            head += "lag %d\n" % lag
        if mode is not None:
            head += "mode %d\n" % mode
        if xcds is not None:
            head += "xcds %d\n" % xcds
        p = subprocess.run([exe, str(workgroups)], input=head + "\n".join(lines) + "\n", capture_output=True,
                           text=True, timeout=120)
        out = p.stdout.strip()
        assert p.returncode == 0 and out.startswith("ok"), out + p.stderr
        _, tasks, tickets, lds, pinned = out.split()
        return int(tasks), int(tickets), int(lds), bool(int(pinned))
    run.exe = exe
    return run


def test_busy_ring_returns_instead_of_waiting(sim):
    """fft3d_batch_submit's slot choice: slots still in flight are skipped,
    never waited for; too few usable slots is reported (the submit then
    returns FFT3D_ERR_BUSY with nothing enqueued)."""
    p = subprocess.run([sim.exe, "ring"], capture_output=True, text=True, timeout=60)
    assert p.returncode == 0 and p.stdout.strip() == "ok ring", p.stdout + p.stderr


def item(shape, dtype, direction, work=1):
    return "%d %d %d %d %d %d" % (shape[0], shape[1], shape[2], 1 if dtype == "f64" else 0, direction, work)


def test_mixed_batch_tables_and_protocol(sim):
    """The 64-field mix: 4 passes per field (2 for fields whose plane step is
    split in the batch: rows + n1 columns each way), every tile inside its
    buffers, the protocol completes on 256 workgroups."""
    mix = fields.batch_mix(64, seed=4)
    tasks, tickets, lds, pinned = sim([item(s, d, 2) for s, d in mix], workgroups=256)
    assert tasks >= 4 * 64 and tickets > 0
    assert lds <= 80 * 1024 - 256
    assert pinned, "64 mixed fields balance over 8 XCDs"
    # the same as one queue
    sim([item(s, d, 2) for s, d in mix], workgroups=256, mode=2)


@pytest.mark.parametrize("lag", [1, 2, 3, 7, 1000])
def test_ticket_orders(sim, lag):
    mix = fields.batch_mix(24, seed=11)
    sim([item(s, d, 2) for s, d in mix], workgroups=32, lag=lag)


def test_every_direction_and_big_shapes(sim):
    """Directions with and without work, degenerate axes, and shapes whose own
    kernels are big-tier (retiled to the small tier in a batch)."""
    shapes = [(1, 1, 2), (2, 3, 4), (1, 8, 16), (8, 1, 8), (12, 9, 24), (96, 96, 96), (128, 128, 128),
              (192, 192, 96), (256, 256, 256), (8, 512, 512), (3, 1024, 1024), (1024, 2, 2), (2, 2048, 16),
              (4, 16, 4096), (729, 4, 6), (512, 512, 512), (4096, 4, 4)]
    lines = []
    for i, s in enumerate(shapes):
        for d in ("f32", "f64"):
            lines.append(item(s, d, i % 3, work=(i // 3) % 2))
    sim(lines, workgroups=96)


def test_random_mixes(sim):
    rng = np.random.default_rng(5)
    ext = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128]
    for trial in range(6):
        lines = []
        for _ in range(int(rng.integers(1, 40))):
            n0, n1 = (int(rng.choice(ext)) for _ in range(2))
            n2 = 2 * int(rng.choice(ext))
            lines.append(item((n0, n1, n2), ("f32", "f64")[int(rng.integers(2))], int(rng.integers(3)),
                              int(rng.integers(2))))
        sim(lines, workgroups=int(rng.integers(1, 200)), lag=int(rng.integers(0, 5)) or None)


def test_one_workgroup_drains_everything(sim):
    """A single workgroup per queue still finishes (every wait is for a
    smaller ticket of the same queue)."""
    three = [item((32, 32, 32), "f32", 2), item((16, 8, 12), "f64", 2), item((8, 8, 8), "f32", 0)]
    sim(three, workgroups=1, mode=2)
    sim(three, workgroups=8, mode=1)


def test_pinning_choice(sim):
    """Auto mode pins items to XCDs only when that balances them: one big
    item among small ones stays on one queue; queue counts follow the XCDs."""
    lop = [item((192, 192, 96), "f64", 2)] + [item((32, 32, 32), "f32", 2)] * 3
    assert not sim(lop, workgroups=64)[3]
    even = [item((64, 64, 64), "f32", 2)] * 16
    assert sim(even, workgroups=64)[3]
    assert sim(even, workgroups=12, xcds=4, mode=1)[3]
    assert not sim(even, workgroups=12, xcds=1)[3]


def test_lost_ticket_state_ends_by_the_iteration_bound(sim):
    """Thread 0's next-ticket word kept where it does not hold its value (LDS
    past the launch's allocation reads zero and drops writes): the ticket loop
    runs ticket 0 again and again.  Without an iteration bound it never ends
    (the simulation gives up and says "unbounded"); with the kernel's bound
    (at most the queue's tickets + 1 iterations) every workgroup leaves and
    the loop error bit is set."""
    items = [item((64, 64, 64), "f32", 2), item((32, 32, 32), "f64", 2)]
    for mode in ("", "mode 2\n"):
        head = mode + "state lost\n"
        p = subprocess.run([sim.exe, "16"], input=head + "\n".join(items) + "\n", capture_output=True, text=True,
                           timeout=120)
        assert p.returncode == 0 and p.stdout.startswith("bounded"), p.stdout + p.stderr
        p = subprocess.run([sim.exe, "16"], input=head + "bound 0\n" + "\n".join(items) + "\n",
                           capture_output=True, text=True, timeout=120)
        assert p.returncode == 3 and p.stdout.startswith("unbounded"), p.stdout + p.stderr


def test_spin_limit_error_path(sim):
    """The kernel's bounded dependency wait with no poll at all (spin 0):
    every dependent task gives up at once, its tiles are skipped, the error
    bit is set and every workgroup still leaves, each ticket taken once."""
    items = [item((64, 64, 64), "f32", 2), item((32, 32, 32), "f64", 2), item((96, 96, 96), "f32", 2)]
    for head in ("spin 0\n", "spin 0\nmode 2\n"):
        p = subprocess.run([sim.exe, "16"], input=head + "\n".join(items) + "\n", capture_output=True, text=True,
                           timeout=120)
        assert p.returncode == 0 and p.stdout.startswith("errbit"), p.stdout + p.stderr
        assert int(p.stdout.split()[1]) > 0
    # a generous limit on the same items: no error, the normal checks
    p = subprocess.run([sim.exe, "16"], input="spin 1000000\n" + "\n".join(items) + "\n", capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 0 and p.stdout.startswith("ok"), p.stdout + p.stderr


def run_levels(sim, lines):
    p = subprocess.run([sim.exe, "1"], input="mode 3\n" + "\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=120)
    out = p.stdout.strip()
    assert p.returncode == 0 and out.startswith("ok levels"), out + p.stderr
    _, _, tasks, launches, tiles, lds = out.split()
    return int(tasks), int(launches), int(tiles), int(lds)


def test_level_mode_schedules(sim):
    """Level mode (one launch per pass level, tile kind, tier and dtype):
    every launch holds one kind, tier and dtype; every item's passes are the
    chain its plan runs alone (fused plane, big-tier ones included, or rows
    + n1 columns; n0 columns), each reading what the one before wrote and in
    a later launch than it; every tile stays inside its item's buffers."""
    mix = fields.batch_mix(64, seed=4)
    tasks, launches, tiles, lds = run_levels(sim, [item(s, d, 2) for s, d in mix])
    # planes larger than the small tier keep their own big-tier fused tile:
    # four passes per field, LDS up to the whole 160 KB
    assert tasks == 4 * 64 and tiles > 0 and lds <= 160 * 1024
    # round trips of fused and split items: at most 8 launches per dtype
    assert launches <= 16
    shapes = [(1, 1, 2), (2, 3, 4), (1, 8, 16), (8, 1, 8), (12, 9, 24), (96, 96, 96), (192, 192, 96),
              (256, 256, 256), (8, 512, 512), (1024, 2, 2), (4, 16, 4096), (729, 4, 6)]
    lines = [item(s, d, i % 3, work=(i // 3) % 2) for i, s in enumerate(shapes) for d in ("f32", "f64")]
    run_levels(sim, lines)
    rng = np.random.default_rng(9)
    ext = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128]
    for trial in range(6):
        lines = []
        for _ in range(int(rng.integers(1, 40))):
            n0, n1 = (int(rng.choice(ext)) for _ in range(2))
            lines.append(item((n0, n1, 2 * int(rng.choice(ext))), ("f32", "f64")[int(rng.integers(2))],
                              int(rng.integers(3)), int(rng.integers(2))))
        run_levels(sim, lines)
