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


def test_multigrid_autotune_leaves_the_state_and_the_cycles_unchanged():
    """autotune_multigrid times whole V-cycles on a scratch copy of the finest
    state: the solver's state is unchanged, every level ends on a tuning it
    accepted, and cycles after tuning are bitwise those of an untuned twin."""
    import torch
    from paper_1710_09995_amd.autotune import MG_CANDIDATES, autotune_multigrid
    from paper_1710_09995_amd.binding import Multigrid, Solver
    case = cases.channel_case(64, 32, 32, mach=0.6, hb=0.05)
    sa, sb = Solver(case), Solver(case)
    ma, mb = Multigrid(sa, 3, 1, 2), Multigrid(sb, 3, 1, 2)
    untuned = [lv.get_tuning() for lv in ma.levels]
    q0 = sa.state()
    res = autotune_multigrid(ma, cycles=5)
    for x, y in zip(sa.state(), q0):
        assert np.array_equal(x, y)
    assert len(res["tunings"]) == 3 and res["ms_per_cycle"] > 0
    allowed = {tuple(c[:3]) for c in MG_CANDIDATES}
    for t, u in zip(res["tunings"], untuned):
        assert (t["kernel"], t["tile_j"], t["tile_k"]) in allowed or t == u
    ha, hb = ma.cycles(4), mb.cycles(4)
    torch.cuda.synchronize()
    assert torch.equal(ha, hb)
    for x, y in zip(sa.state(), sb.state()):
        assert np.array_equal(x, y)
    for m in (ma, mb):
        m.close()
    sa.close()
    sb.close()
