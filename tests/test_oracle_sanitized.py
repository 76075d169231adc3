"""The oracle's CPU pins once more against a build instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (halting on the first report):
out-of-bounds accesses, use after free, signed overflow, misaligned or null
dereferences and the like anywhere in the oracle's C make this test fail."""
import os

import pytest

from oracle import build as oracle_build

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = ["test_oracle_rng.py", "test_oracle_estimator.py", "test_oracle_smc.py", "test_oracle_paper_schemes.py",
         "test_oracle_move_pins.py"]


def test_oracle_pins_pass_under_address_and_undefined_behaviour_sanitizers():
    if not os.path.exists(os.popen("gcc -print-file-name=libasan.so").read().strip()):
        pytest.skip("no libasan for gcc on this machine")
    rc = oracle_build.run_sanitized_tests(tuple(os.path.join(HERE, f) for f in FILES) + ("-q", "-p", "no:cacheprovider"))
    assert rc == 0
