"""The oracle against its own stored output on a tiny seeded case
(tests/golden/oracle_small.json, written by tests/golden/make_oracle_fixture.py
from the oracle alone). Not a pin of the method (the pins are in
test_oracle_pins.py; the paper prints no worked example to store): it makes
any change to the oracle's arithmetic visible, so that such a change is made
on purpose and justified when the fixture is rewritten."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _generator():
    spec = importlib.util.spec_from_file_location(
        "make_oracle_fixture", os.path.join(GOLDEN, "make_oracle_fixture.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_reproduces_its_stored_output():
    stored = json.load(open(os.path.join(GOLDEN, "oracle_small.json")))["cases"]
    now = _generator().compute()
    assert set(now) == set(stored)
    for medium, ref in stored.items():
        got = now[medium]
        assert got["bins"] == ref["bins"], medium                   # bins exactly
        np.testing.assert_allclose(got["t"], ref["t"], rtol=1e-15, atol=0, err_msg=medium)
        for f in ("endpoint", "zhs"):
            assert got[f]["index"] == ref[f]["index"], (medium, f)   # same nonzero bins
            np.testing.assert_allclose(got[f]["value"], ref[f]["value"], rtol=1e-12, atol=0,
                                       err_msg=f"{medium} {f}")
