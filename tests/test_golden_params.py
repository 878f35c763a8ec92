"""The default parameters match the values the paper states (tests/golden/params.json)."""
import json
import os

import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "params.json")))


@pytest.mark.parametrize("name", ["kappa1", "kappa2", "eta", "ko_sigma", "shift_coeff"])
def test_oracle_defaults(oz, name):
    assert getattr(oz.params(), name) == GOLDEN[name]["value"]


def test_courant_factor_in_workloads():
    from paper_2607_08743_amd import inputs as I
    for g, _, dt in (I.config_plane_wave(), I.config_punctures(16)):
        assert dt == GOLDEN["courant"]["value"] * g.h[0]
    for box in I.config_hierarchy(sizes=(8, 8)):
        assert box.dt == GOLDEN["courant"]["value"] * box.grid.h[0]
