"""The context's simulation bookkeeping, checked on the CPU under
AddressSanitizer and UndefinedBehaviorSanitizer: a context destroys the
simulations still created on it exactly once, a destroyed simulation leaves
every list (no use after free at the next synchronisation), and a sticky abort
flag marks every simulation advanced by a persistent launch since the last
synchronising call, even when a later launch finished cleanly."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_registry_under_sanitizers():
    src = os.path.join(HERE, "native", "registry_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "registry_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-o", exe, src]
        try:
            subprocess.run(cmd, check=True, capture_output=True, text=True)
        except FileNotFoundError:
            pytest.skip("g++ is not installed")
        except subprocess.CalledProcessError as e:
            if "asan" in (e.stderr or "").lower():
                pytest.skip("gcc's AddressSanitizer runtime is not installed")
            raise AssertionError(e.stderr)
        res = subprocess.run([exe], capture_output=True, text=True, timeout=60,
                             env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "registry ok" in res.stdout, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
