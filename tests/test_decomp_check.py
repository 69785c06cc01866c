"""The library's block-independence check (Sec. 2.1, remark after eq.
gendecomp), which marks only the blocks' boundary rows and columns, gives the
verdict of a check that marks every site of every block and its neighbours, on
a sweep of lattice and block shapes, colour maps and both event kinds; built
and run on the CPU under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_boundary_check_equals_every_site_check():
    src = os.path.join(HERE, "native", "decomp_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "decomp_check")
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
        res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "decomposition ok" in res.stdout, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
