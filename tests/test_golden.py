"""CPU checks of the stored oracle samples used by the full-size GPU parity
tests: each was written by tests/golden/make_golden.py from the oracle only,
and its rows reach the levels of the library's dissection that matter -- the
top separator (the largest front), a separator below it, and an innermost
domain -- so that every level of the selected inversion is compared."""
import json
import os

import numpy as np
import pytest

import paper_1005_0088_amd as nd
from synth import config_system

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _levels_of_rows(sysd, rows):
    P = nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["coords"], 32, cell=sysd["cell"])
    ex = P.export()
    pos = np.empty(sysd["n"], np.int64)
    pos[ex["perm"]] = np.arange(sysd["n"])
    out = []
    for r in rows:
        f = int(np.searchsorted(ex["j0"], pos[r], side="right") - 1)
        out.append((int(ex["depth"][f]), bool(np.any(ex["parent"] == f))))
    return out


def _check_strata(sysd, rows):
    lv = _levels_of_rows(sysd, rows)
    assert any(d == 0 for d, _ in lv), "no row in the top separator"
    assert any(d >= 1 and sep for d, sep in lv), "no row in a lower separator"
    assert any(not sep for _, sep in lv), "no row in an innermost domain"


def _load(name):
    path = os.path.join(GOLDEN, "rho_sampled_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("no stored sample for %s" % name)
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["square2d_64x4", "cubic3d_24x4", "cubic3d_40x4"])
def test_sample_rows_span_the_dissection_levels(name):
    g = _load(name)
    sysd = config_system(name)
    _check_strata(sysd, g["rows"])
    # every stored entry belongs to a sampled row
    rows_of = np.repeat(np.arange(sysd["n"]), np.diff(sysd["row_ptr"]))
    assert set(rows_of[np.asarray(g["entries"])].tolist()) == set(g["rows"])


def test_eight_lattice_sample_spans_the_levels_of_every_member():
    g = _load("multi2d_8x4")
    assert [m["dims"] for m in g["members"]] == [[k, k] for k in (32, 40, 48, 56, 64, 72, 80, 96)]
    assert g["n_poles"] == 100
    for i, m in enumerate(g["members"]):
        _check_strata(config_system("multi2d_8x4", i), m["rows"])


@pytest.mark.parametrize("name", ["square2d_64x4", "cubic3d_24x4"])
def test_periodic_sample_rows_span_the_dissection_levels(name):
    g = _load(name + "_periodic")
    sysd = config_system(name, periodic=True)
    assert g["cell"] == sysd["cell"]
    _check_strata(sysd, g["rows"])
    rows_of = np.repeat(np.arange(sysd["n"]), np.diff(sysd["row_ptr"]))
    assert set(rows_of[np.asarray(g["entries"])].tolist()) == set(g["rows"])
