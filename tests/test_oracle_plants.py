"""The oracle's pins have teeth: a variant of the oracle built with one
plausible mistake (a wrong sign, a dropped guard, a wrong neighbour index, a
wrong half step, a wrong factor, a missing colour test, a wrong constant, a
wrong key schedule, a transposed direction, a colour
drawn at the wrong rate, an off-by-one quantile, a wrong neighbour count) must fail at least one pin.

Each variant is compiled on the CPU into a temporary library and the relevant
pin tests are run against it in a child process."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

PLANTS = {
    1: ("spin-flip rate with the sign of the exponent flipped",
        ["test_oracle_serial.py::test_serial_matches_master_equation"]),
    2: ("Philox key bumped before the first round",
        ["test_oracle_rng.py::test_philox_vs_aten"]),
    3: ("descent subtracting the right child instead of the left",
        ["test_oracle_tree.py"]),
    4: ("Strang middle window of length dt/2 instead of dt",
        ["test_oracle_fs.py::test_schedule_window_lists", "test_oracle_fs.py::test_schedule_orders_of_accuracy"]),
    5: ("-y neighbour taken as +y",
        ["test_oracle_serial.py::test_serial_matches_master_equation"]),
    6: ("A+B reaction rate k_r/2 per direction instead of k_r/4",
        ["test_oracle_rates.py::test_zgb_table_vs_event_enumeration"]),
    7: ("every block active in every window (colour ignored)",
        ["test_oracle_fs.py::test_fs_matches_split_propagator"]),
    8: ("wrong sign of the low part of ln 2",
        ["test_oracle_rng.py::test_log_special_values", "test_oracle_rng.py::test_log_accuracy_on_uniforms"]),
    9: ("pair partner direction from the channel group instead of the direction",
        ["test_oracle_serial.py::test_serial_matches_master_equation"]),
    10: ("random schedule drawing one colour per step instead of per window",
         ["test_oracle_fs.py::test_random_schedule_colours_uniform_and_independent",
          "test_oracle_fs.py::test_fs_random_schedule_matches_averaged_propagator"]),
    11: ("workload quantile one block late (strict instead of non-strict CDF test)",
         ["test_oracle_balance.py"]),
    12: ("exchange barrier counting the empty neighbours instead of the occupied ones",
         ["test_oracle_kawasaki.py::test_serial_matches_master_equation"]),
    13: ("nested inner schedule spanning dt instead of the outer window's length",
         ["test_oracle_nested.py::test_window_lists_by_hand"]),
}


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=[PLANTS[k][0] for k in sorted(PLANTS)])
def test_planted_mistake_is_caught(plant):
    import oracle
    desc, tests = PLANTS[plant]
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, f"liboracle_plant{plant}.so")
        oracle.build(out=lib, defines=[f"OR_PLANT={plant}"])
        env = dict(os.environ, FSKMC_ORACLE_LIB=lib, FSKMC_ORACLE_PLANT=str(plant), PYTHONPATH=ROOT)
        args = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
        args += [os.path.join(HERE, t) for t in tests]
        res = subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert res.returncode != 0, f"planted mistake {plant} ({desc}) passed every pin:\n{res.stdout[-2000:]}"
        assert "failed" in res.stdout, res.stdout[-2000:]
