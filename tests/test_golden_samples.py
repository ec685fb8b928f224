"""Consistency of the stored full-size sample fixtures (written by
tests/golden/make_samples.py from the oracle's direct solve): the fields
the full-size GPU parity tests rely on."""
import json
import os

import numpy as np
import pytest


@pytest.mark.parametrize("name,ndofs", [("level10_traction_samples.json", 2 * 4 ** 10),
                                        ("lshape9_samples.json", 2 * 3 * 4 ** 9)])
def test_sample_fixture_is_consistent(name, ndofs):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))
    idx = np.asarray(g["index"])
    val = np.asarray(g["value"])
    assert g["ndofs"] == ndofs
    assert idx.size == val.size == len(g["stratum"]) > 2048
    strata = set(g["stratum"])
    assert {"uniform", "clamped_edge", "loaded_edge"} <= strata
    assert ("reentrant_corner" in strata) == name.startswith("lshape")
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < g["ndofs"]
    # the samples are part of the whole vector
    assert float(val @ val) <= g["norm2"]
    assert np.abs(val).max() <= g["max_abs"]
    # <f, u*> = <u*, K u*> > 0 for K SPD and a nonzero load
    assert g["f_dot_u"] > 0.0
