"""Oracle regression fixtures (tests/golden/oracle_values.json, written by
tests/golden/make_golden.py from the oracle alone): a change of the oracle's
arithmetic must show up here."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_its_frozen_values():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(HERE, "golden", "oracle_values.json")) as fh:
        ref = json.load(fh)
    got = mod.build()
    assert got["philox_words"] == ref["philox_words"]
    for key in ("ttbar_integrand_pb", "drellyan_integrand_pb", "singletop_integrand_pb"):
        assert got[key] == pytest.approx(ref[key], rel=1e-13, abs=0)
    for key in ("mean", "sigma", "chi2_dof"):
        assert got["vegas_gauss4_3x20000"][key] == pytest.approx(ref["vegas_gauss4_3x20000"][key], rel=1e-12)
