"""Pins for the oracle's random numbers and logarithm (test infrastructure).

* Philox4x32-10 (Salmon et al., SC'11) must equal two independent open-source
  implementations present in this image: rocRAND's header and PyTorch's ATen
  header, each compiled into a small comparator program.
* The uniforms U in (0,1], V in [0,1) follow from the 53-bit conversion.
* The logarithm must be within 2 ulp of a 40-digit decimal logarithm and exact
  at 1 and at powers of two (up to the ln 2 split).
"""
import math
import os
import shutil
import subprocess
import tempfile
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
TORCH_INC = None
try:
    import torch.utils.cpp_extension as _ce
    TORCH_INC = _ce.include_paths()[0]
except Exception:  # pragma: no cover
    pass


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    words = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    edge = np.array([[0, 0, 0, 0, 0, 0],
                     [0xFFFFFFFF] * 6,
                     [1, 0, 0, 0, 0, 0],
                     [0, 0, 0, 0, 0xFFFFFFFF, 0],
                     [5, 7, 11, 0, 0, 3],
                     [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 2, 0, 0]], dtype=np.uint64)
    return np.concatenate([edge, words]).astype(np.uint64)


def _run_comparator(exe, inp):
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in inp) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def _oracle_blocks(orc, inp):
    return np.array([orc.philox(r[:4], r[4:]) for r in inp], dtype=np.uint64)


@pytest.fixture(scope="module")
def tmpdir_mod():
    d = tempfile.mkdtemp(prefix="philox_cmp_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_philox_vs_aten(orc, tmpdir_mod):
    if TORCH_INC is None or shutil.which("g++") is None:
        pytest.skip("torch headers or g++ unavailable")
    exe = os.path.join(tmpdir_mod, "aten")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", TORCH_INC, "-o", exe,
                           os.path.join(HERE, "comparators", "philox_aten.cpp")])
    inp = _inputs(3000, 1)
    np.testing.assert_array_equal(_run_comparator(exe, inp), _oracle_blocks(orc, inp))


def test_philox_vs_rocrand(orc, tmpdir_mod):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc unavailable")
    exe = os.path.join(tmpdir_mod, "rocrand")
    subprocess.check_call([hipcc, "--cuda-host-only", "-O1", "-std=c++17", "-w", "-o", exe,
                           os.path.join(HERE, "comparators", "philox_rocrand.cpp")])
    inp = _inputs(3000, 2)
    np.testing.assert_array_equal(_run_comparator(exe, inp), _oracle_blocks(orc, inp))


def test_uniform_conversion(orc):
    U, V = orc.uniforms([0, 0, 0, 0])
    assert U == 2.0 ** -53 and V == 0.0
    U, V = orc.uniforms([0xFFFFFFFF] * 4)
    assert U == 1.0 and V == 1.0 - 2.0 ** -53
    # top 53 bits of the 64-bit word: the lowest 11 bits are ignored
    U, V = orc.uniforms([0, 0x7FF, 0, 0x800])
    assert U == 2.0 ** -53 and V == 2.0 ** -53
    U, V = orc.uniforms([0x80000000, 0, 0x80000000, 0])
    assert U == 0.5 + 2.0 ** -53 and V == 0.5


def _ulp_err(got, u):
    exact = Decimal(u).ln()
    ref = float(exact)
    return float(abs(Decimal(got) - exact) / Decimal(math.ulp(ref))) if ref != 0 else abs(got)


def test_log_special_values(orc):
    assert orc.log(1.0) == 0.0
    assert math.copysign(1.0, orc.log(1.0)) == 1.0
    for e in (1, 2, 10, 52, 53, 100, 1022):
        assert _ulp_err(orc.log(2.0 ** -e), 2.0 ** -e) <= 1.0
    # smallest uniform the generator produces, and a subnormal input
    assert _ulp_err(orc.log(2.0 ** -53), 2.0 ** -53) <= 1.0
    assert _ulp_err(orc.log(5e-324), 5e-324) <= 1.0


def test_log_accuracy_on_uniforms(orc):
    getcontext().prec = 40
    rng = np.random.default_rng(7)
    k = rng.integers(0, 2 ** 53, size=30000, dtype=np.uint64)
    us = [(int(v) + 1) * 2.0 ** -53 for v in k]
    # values near 1 (tiny |log|) and near the sqrt(2) split point
    us += [1.0 - i * 2.0 ** -53 for i in range(1, 400)]
    us += [math.sqrt(0.5) * (1 + i * 2.0 ** -50) for i in range(-200, 200)]
    us += [math.sqrt(0.5) * 2 ** -j for j in range(1, 40)]
    worst = 0.0
    for u in us:
        if not (0.0 < u <= 1.0):
            continue
        worst = max(worst, _ulp_err(orc.log(u), u))
    assert worst <= 2.0, worst


def test_log_monotone_near_one(orc):
    prev = orc.log(1.0)
    for i in range(1, 2000):
        cur = orc.log(1.0 - i * 2.0 ** -53)
        assert cur <= prev
        prev = cur
