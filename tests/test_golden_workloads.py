"""Workload shapes the paper prints, held as fixtures under tests/golden/."""
import json
import os

import numpy as np

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_fig2a_generator_matches_paper_shape():
    g = _load("fig2a_workload.json")
    c = datagen.fig2a_case()
    assert c["counts"].size == g["nbins"]
    assert tuple(c["range"]) == (g["lo"], g["hi"])
    assert int(c["counts"].sum()) == g["entries"]
    np.testing.assert_array_equal(c["theta0"], g["gaus_params"])


def test_listing1_launch_shape():
    g = _load("listing1_launch.json")
    assert g["N"] // g["block"] + 1 == g["grid"]
    assert g["grid"] * g["block"] >= g["N"]
