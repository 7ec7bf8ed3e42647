"""The oracle reproduces its stored regression results exactly
(tests/golden/oracle_regression.json, written by tests/golden/make_golden.py
from the oracle alone).  A change of the oracle's arithmetic must regenerate
the file in the same commit and name the passage of the paper that
justifies it."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402

with open(os.path.join(HERE, "golden", "oracle_regression.json")) as f:
    GOLDEN = json.load(f)


@pytest.mark.parametrize("name,wl", list(make_golden.cases()), ids=lambda x: x if
                         isinstance(x, str) else "")
def test_oracle_matches_stored_results(name, wl):
    assert make_golden.summarise(wl) == GOLDEN[name]
