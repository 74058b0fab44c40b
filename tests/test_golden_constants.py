"""The default parameters of the oracle and of the library against the
constants the paper states (tests/golden/paper_constants.json, each entry
with where the paper states it).  pdlp_params_default is host code: the
library loads and answers without a GPU."""
import json
import os

import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _constants(params_only=True):
    with open(GOLDEN) as f:
        cs = json.load(f)["constants"]
    return [c for c in cs if c.get("param", True)] if params_only else cs


def constant(key):
    """Value of a constant of the golden file by key."""
    return next(c["value"] for c in _constants(False) if c["key"] == key)


@pytest.mark.parametrize("c", _constants(), ids=lambda c: c["key"])
def test_oracle_defaults_are_the_papers(c):
    assert getattr(oracle.Params(), c["key"]) == c["value"], c["where"]


@pytest.mark.parametrize("c", _constants(), ids=lambda c: c["key"])
def test_library_defaults_are_the_papers(c):
    pd = pytest.importorskip("paper_2501_07018_amd")
    try:
        p = pd.pdlp_params_default()
    except ImportError:
        pytest.skip("libpdlp.so is not built")
    assert getattr(p, c["c_field"]) == c["value"], c["where"]
    assert p.pock_chambolle == 1
