"""The oracle reproduces its stored results on tests/golden/tiny_epoch.json (written by
tests/golden/make_golden.py from the oracle alone): a change of the oracle's arithmetic shows up here."""
import json
import os

import numpy as np

from tests.golden.make_golden import oracle_results

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_stored_golden():
    stored = json.load(open(os.path.join(HERE, "tiny_epoch.json")))
    now = oracle_results(stored["case"])
    for kind in ("exact", "relaxed"):
        for key in ("A", "B"):
            for a, b in zip(now[kind][key], stored[kind][key]):
                np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(now[kind]["loss"], stored[kind]["loss"], rtol=1e-12)
