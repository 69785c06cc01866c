"""The oracle's C and libfskmc's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The oracle is rebuilt with gcc -fsanitize=address,undefined and a set of its
pins runs against that build in a child process; libfskmc is rebuilt with
the sanitizers on its host code only (-Xarch_host before each -fsanitize=;
the gfx950 code is unchanged) and the host-side tests run against it.  Any
report fails the child (UBSan halts on the first error)."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _child(tests, env_extra):
    env = dict(os.environ, PYTHONPATH=ROOT, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    args = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + [os.path.join(HERE, t) for t in tests]
    return subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def _runtime(cmd):
    try:
        path = subprocess.run(cmd, capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan():
    import oracle
    asan = _runtime(["gcc", "-print-file-name=libasan.so"])
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_asan.so")
        oracle.build(out=lib, extra_flags=["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                           "-fno-omit-frame-pointer", "-O1"])
        res = _child(["test_oracle_rng.py", "test_oracle_tree.py", "test_oracle_rates.py",
                      "test_oracle_fs.py::test_schedule_window_lists", "test_oracle_fs.py::test_fs_matches_split_propagator",
                      "test_oracle_kawasaki.py::test_rate_table_vs_event_enumeration",
                      "test_oracle_kawasaki.py::test_particle_number_conserved", "test_oracle_nested.py"],
                     {"FSKMC_ORACLE_LIB": lib, "LD_PRELOAD": asan})
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "passed" in res.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_host_library_under_asan_and_ubsan():
    from paper_1105_4673_amd import build
    rt = _runtime([build.HIPCC.replace("hipcc", "amdclang++"), "-print-file-name=libclang_rt.asan-x86_64.so"])
    if rt is None:
        rt = _runtime(["/opt/rocm/lib/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libfskmc_asan.so")
        build.build(out=lib, extra_flags=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                          "-Xarch_host", "-fno-sanitize-recover=undefined",
                                          "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"])
        res = _child(["test_host_errors.py", "test_balance_partition.py"], {"FSKMC_LIB": lib, "LD_PRELOAD": rt})
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "passed" in res.stdout, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
