"""The CPU oracle against closed forms, invariants, library routines and
brute force (no GPU needed)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("check", P.ALL, ids=[c.__name__ for c in P.ALL])
def test_oracle_pin(orc, check):
    check()


def test_pyr_down_direct_form(orc):
    P.check_pyr_down_library(direct=True)
