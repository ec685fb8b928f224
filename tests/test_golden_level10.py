"""Consistency of the stored level-10 sample fixture (written by
tests/golden/make_level10_samples.py from the oracle's direct solve): the
fields the level-10 GPU parity test relies on."""
import json
import os

import numpy as np


def test_level10_fixture_is_consistent():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "level10_traction_samples.json")))
    idx = np.asarray(g["index"])
    val = np.asarray(g["value"])
    assert g["ndofs"] == 2 * 4 ** 10
    assert idx.size == val.size == 2048
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < g["ndofs"]
    # the samples are part of the whole vector
    assert float(val @ val) <= g["norm2"]
    assert np.abs(val).max() <= g["max_abs"]
    # <f, u*> = <u*, K u*> > 0 for K SPD and a nonzero load
    assert g["f_dot_u"] > 0.0
