"""Each planted mistake in the oracle must fail at least one pin.

The oracle source carries a few ``ORC_MUTANT_*`` switches; each compiles a copy of the oracle
with one plausible slip (a wrong sign, a dropped power, a dropped coordinate, a skipped
substitution, the wrong tie rule, a level that restarts from the input instead of the residual,
an unweighted volume update, a wrong coefficient or power in a Table 1 function). This shows the pins are strong enough to catch them.
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = ["ORC_MUTANT_PHI_SIGN", "ORC_MUTANT_PHI_POWER", "ORC_MUTANT_DIST_DROP_Z",
           "ORC_MUTANT_NO_BACKSOLVE", "ORC_MUTANT_ERROR_SIGN", "ORC_MUTANT_TIE_HIGH",
           "ORC_MUTANT_LEVEL_RESTART", "ORC_MUTANT_PSI_SKIP", "ORC_MUTANT_C4_COEF",
           "ORC_MUTANT_C6_POWER"]


@pytest.mark.parametrize("mutant", MUTANTS)
def test_planted_mistake_is_caught(tmp_path, mutant):
    path = os.path.join(str(tmp_path), f"liborc_{mutant.lower()}.so")
    oracle.build(path, defines=[mutant])
    o = oracle.Oracle(path)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except (AssertionError, RuntimeError, FloatingPointError, ValueError,
                __import__("numpy").linalg.LinAlgError) as e:  # noqa: F841
            failed.append(pin.__name__)
    assert failed, f"{mutant} passed every pin"
