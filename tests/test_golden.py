"""The oracle against its regression fixture (tests/golden/oracle_small.json, written by
tests/golden/make_golden.py from the oracle alone): two steps of a small bending vesicle in
Poiseuille flow and of a Cahn-Hilliard droplet in Couette flow. A change of the oracle's
arithmetic shows up here; the fixture is rewritten only with a change whose commit names the
passage of the paper that justifies it."""
import importlib.util
import json
import os

import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _make_golden():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("case", ["bending_poiseuille", "ch_couette"])
def test_oracle_matches_fixture(case):
    mg = _make_golden()
    stored = json.load(open(os.path.join(HERE, "oracle_small.json")))
    assert stored["nsteps"] == mg.NSTEPS
    spec = stored["cases"][case]["spec"]
    want = stored["cases"][case]["result"]
    got = mg.summary(mg.oracle_run(mg.case_workload(spec)))
    for k, v in want["scalars"].items():
        assert got["scalars"][k] == pytest.approx(v, rel=1e-12, abs=1e-14), k
    for field in (f for f in want if f != "scalars"):
        assert got[field]["l2"] == pytest.approx(want[field]["l2"], rel=1e-12), field
        assert got[field]["sum"] == pytest.approx(want[field]["sum"], rel=1e-10, abs=1e-12), field
        assert got[field]["samples"] == pytest.approx(want[field]["samples"], rel=1e-11, abs=1e-14), field
