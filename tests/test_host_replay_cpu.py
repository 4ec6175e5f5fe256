"""Host side of the library under AddressSanitizer / UndefinedBehaviorSanitizer
(no GPU needed): the library's sources are built against a checking stand-in
for the HIP runtime (tests/cpu_runtime), and the C-ABI call sequences of the
GPU tests are replayed (tests/cpu_runtime/replay.py).  Every copy is checked
against the allocations it names, every launch against the kernel's limits,
every stream / event / graph / BLAS handle against the live ones, and the
library's own table checks run at plan, pool and batch creation.

Regression pinned here: destroying a pool after its plan used to read the
freed plan (heap-use-after-free found by this replay); the pool is now
detached and refuses to run.

The kernel-executing build (tests/cpu_runtime/kexec) goes further: the
kernels themselves run on the host, one fiber per work-item, so GPU test
cases run end to end on the CPU with every kernel access to device memory
and to its dynamic LDS checked by AddressSanitizer, and their results are
compared with the oracle by the test's own assertions.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RT = os.path.join(ROOT, "tests", "cpu_runtime")


@pytest.fixture(scope="module")
def hostcheck():
    if shutil.which("/opt/rocm/bin/hipcc") is None:
        pytest.skip("hipcc is not installed")
    sys.path.insert(0, RT)
    import build as rt_build  # tests/cpu_runtime/build.py
    rt_build.build()
    return rt_build.asan_runtime()


def _replay(asan, *suites, timeout=900, busy_streams=False):
    env = dict(os.environ)
    if busy_streams:  # every stream query reports pending work, so the calls' fences run
        env["FSV_STUB_BUSY_STREAMS"] = "1"
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(RT, "replay.py"), *suites], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=timeout)
    tail = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, tail
    assert "replay done" in r.stdout and "AddressSanitizer" not in r.stderr, tail
    return r.stdout


def test_replay_sigma_path_sequences(hostcheck):
    # the nine alpha-beta path cases (direct, factorised, automatic choice on
    # integrals of rank 8, 12 and 28) on both engines, as the GPU test runs them
    out = _replay(hostcheck, "sigma")
    assert out.count("sigma paths") == 9


def test_replay_pools_and_lifetimes(hostcheck):
    # pools of both kinds, a pool destroyed after its plan, initial-state calls
    _replay(hostcheck, "pools")


def test_replay_batches(hostcheck):
    _replay(hostcheck, "batch")


def test_replay_xcd_placement(hostcheck):
    # a 20-qubit plan whose packet runs are placed by XCD: equal XCD ranges
    # (packet counts multiples of 8), programs checked, calls replayed
    out = _replay(hostcheck, "placement")
    assert "placement" in out


def test_replay_with_busy_streams(hostcheck):
    # the calls skip their stream fences when a stream is idle; here no stream
    # is ever idle, so every fence's event record and wait are exercised
    _replay(hostcheck, "pools", "batch", busy_streams=True)


@pytest.fixture(scope="module")
def kexec(hostcheck):
    import build as rt_build  # tests/cpu_runtime/build.py
    rt_build.build_kexec()
    return hostcheck


def _gpu_tests_on_cpu(asan, *selection, timeout=1200):
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", FSV_STUB_LIB="kexec", FSV_STUB_RUN_SKIPPED="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "tests.cpu_runtime.stub_plugin",
                        "-p", "no:cacheprovider", *selection], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=timeout)
    tail = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    return r.stdout


def test_kernels_on_cpu_sigma_paths(kexec):
    # the alpha-beta product directly, through the rank-8 factors (forced) and
    # by the automatic choice, on both engines: the case after which the GPU
    # test process aborted, with its kernels run under AddressSanitizer
    out = _gpu_tests_on_cpu(kexec, "tests/test_gpu_parity.py::test_sigma_paths", "-k", "8-")
    assert "3 passed" in out


def test_kernels_on_cpu_energy_c2(kexec):
    # packet runs, the same-spin GEMM and the factorised product inside
    # captured graphs, replayed
    out = _gpu_tests_on_cpu(kexec, "tests/test_gpu_parity.py::test_energy_small_configs[0-C2]")
    assert "1 passed" in out
