"""Memory safety of the library on the CPU: its own sources, built against a CPU stand-in for the
HIP runtime with AddressSanitizer (tests/memcheck), driven through the C ABI on small boxes.  Any
out-of-bounds or null access in the host logic or in a kernel aborts the run with a report.

This is not a parity test (those run on the GPU); it checks that every access stays inside its
buffer for the call sequences in tests/memcheck/sequence.py."""

import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "memcheck"))


@pytest.fixture(scope="module")
def memcheck_lib(tmp_path_factory):
    import build as mbuild

    try:
        asan = mbuild.asan_runtime()
    except Exception as e:  # pragma: no cover
        pytest.skip(f"no g++ AddressSanitizer runtime: {e}")
    if not os.path.exists(asan):
        pytest.skip("no g++ AddressSanitizer runtime")
    return mbuild.build(str(tmp_path_factory.mktemp("memcheck"))), asan


@pytest.mark.parametrize("part", ["solver", "network", "p1", "sphere", "mixed"])
def test_call_sequences_stay_in_bounds(memcheck_lib, part):
    lib, asan = memcheck_lib
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:redzone=128",
               OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    res = subprocess.run([sys.executable, os.path.join(HERE, "memcheck", "sequence.py"), lib, part],
                         capture_output=True, text=True, env=env, timeout=900)
    print(res.stdout)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-6000:]
    assert "sequence complete" in res.stdout
