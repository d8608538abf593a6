"""GPU: the tile autotuner picks a valid tuning, leaves the solver state
unchanged, and the chosen tuning gives the same bits as the simple kernel."""
import numpy as np
import pytest

from paper_1710_09995_amd import cases

pytestmark = pytest.mark.gpu


def test_autotune_valid_and_bitwise(tmp_path, monkeypatch):
    from paper_1710_09995_amd.autotune import autotune
    from paper_1710_09995_amd.binding import Solver
    monkeypatch.setenv("CFD_TUNE_CACHE", str(tmp_path / "tune.json"))
    case = cases.bump_ns_case(70, 20, 12, seed=3, noise=1e-3, reynolds=5e3)
    s = Solver(case)
    before = s.state()
    res = autotune(s, candidates=[(0, 2, 4, 0), (0, 4, 8, 1), (0, 8, 16, 0)], steps=2, verify=True)
    assert res["tuning"]["kernel"] == 0 and not res["cached"]
    after = s.state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    res2 = autotune(s, candidates=[(0, 2, 4)], steps=1)
    assert res2["cached"] and res2["tuning"] == res["tuning"]
    s.close()
