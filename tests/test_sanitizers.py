"""Host code under the sanitizers (CPU only).

* oracle/oracle.c with AddressSanitizer + UndefinedBehaviorSanitizer (gcc),
  driven by tests/oracle_sanitize.c: every entry point on small shapes.
* The library's host C++ (plans, tunings, the tuning-table reader, the C
  interface, the server in its no-device mode) with ASan + UBSan (g++),
  driven by tests/host_sanitize.cpp, the device half replaced by
  tests/host_stubs.cpp.
* The server's threads (dispatcher and four client threads) and the batched
  kernel's ticket protocol simulated on host threads (tests/batch_sim.cpp)
  with ThreadSanitizer.  TSan builds use ROCm's clang: the gcc 11 TSan
  runtime does not intercept pthread_cond_clockwait, which
  std::condition_variable::wait_for uses, and reports a false double lock.
Every run must exit 0 with no sanitizer report."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1406_5597_amd", "csrc")
HOST_SRC = [os.path.join(CSRC, f) for f in ("fft3d_abi.cpp", "fft3d_plan.cpp", "fft3d_tune.cpp",
                                             "fft3d_batch_host.cpp", "fft3d_server.cpp", "fft3d_dispatch.cpp")]
HIP = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
       "-L/opt/rocm/lib", "-lamdhip64", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]
ASAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
TSAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=thread"]
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           TSAN_OPTIONS="halt_on_error=1", OMP_NUM_THREADS="4")


def build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "build failed: %s\n%s" % (" ".join(cmd), r.stderr[-3000:])


def run(args, stdin=None, timeout=600):
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, input=stdin, timeout=timeout)
    report = r.stderr + r.stdout
    assert r.returncode == 0, report[-4000:]
    for word in ("AddressSanitizer", "runtime error", "ThreadSanitizer", "LeakSanitizer"):
        assert word not in report, report[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return tmp_path_factory.mktemp("san")


def test_oracle_asan_ubsan(outdir):
    exe = str(outdir / "oracle_asan")
    build(["gcc", "-std=c11"] + ASAN + ["-fopenmp", os.path.join(ROOT, "tests", "oracle_sanitize.c"),
                                        os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    assert run([exe]).strip() == "ok oracle"


@pytest.fixture(scope="module")
def host_asan(outdir):
    exe = str(outdir / "host_asan")
    build(["g++", "-std=c++17"] + ASAN + [os.path.join(ROOT, "tests", "host_sanitize.cpp"),
                                          os.path.join(ROOT, "tests", "host_stubs.cpp")] + HOST_SRC + HIP +
          ["-o", exe])
    return exe


def test_plans_asan_ubsan(host_asan):
    assert run([host_asan, "plans"]).strip() == "ok plans"


def test_tuning_table_reader_asan_ubsan(host_asan, outdir):
    d = outdir / "table"
    d.mkdir()
    assert run([host_asan, "table", str(d)]).strip() == "ok table"


def test_server_asan_ubsan(host_asan):
    assert run([host_asan, "server"]).strip() == "ok server"


def test_server_threads_tsan(outdir):
    exe = str(outdir / "host_tsan")
    build([CLANG, "-std=c++17"] + TSAN + [os.path.join(ROOT, "tests", "host_sanitize.cpp"),
                                          os.path.join(ROOT, "tests", "host_stubs.cpp")] + HOST_SRC + HIP +
          ["-o", exe])
    for _ in range(3):
        assert run([exe, "server"]).strip() == "ok server"


def test_batch_protocol_tsan_and_asan(outdir):
    """The ticket protocol on host threads (32 workgroups, pinned and spread
    queues) with ThreadSanitizer, and the task-list builder with ASan."""
    src = [os.path.join(ROOT, "tests", "batch_sim.cpp"), os.path.join(CSRC, "fft3d_plan.cpp"),
           os.path.join(CSRC, "fft3d_batch_host.cpp")]
    items = "\n".join(["32 32 32 0 2 1", "48 48 48 1 2 1", "64 64 64 0 0 1", "16 16 16 1 1 0",
                       "96 96 96 0 2 1", "192 192 96 1 2 1", "128 128 128 0 1 1", "256 256 256 0 2 1"]) + "\n"
    t = str(outdir / "batch_tsan")
    build([CLANG, "-std=c++17"] + TSAN + src + HIP + ["-o", t])
    a = str(outdir / "batch_asan")
    build(["g++", "-std=c++17"] + ASAN + src + HIP + ["-o", a])
    for exe in (t, a):
        for head in ("", "mode 1\n", "mode 2\n", "lag 1\n"):
            assert run([exe, "32"], stdin=head + items).startswith("ok")
        assert run([exe, "ring"]).strip() == "ok ring"
