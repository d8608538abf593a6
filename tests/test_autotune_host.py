"""Host logic of the multigrid autotuner (autotune_multigrid) on stand-in
objects: per level, from the finest, it keeps the candidate whose whole
cycles time fastest, skips candidates a level refuses, times on a scratch
arena (never on the solver's state) and leaves every level on its pick."""
from paper_1710_09995_amd.autotune import autotune_multigrid


class _Clock:
    now = 0.0


class _Event:
    def __init__(self, **kw):
        self.t = None

    def record(self, stream):
        self.t = _Clock.now

    def elapsed_time(self, other):
        return other.t - self.t


class _Cuda:
    Event = _Event

    @staticmethod
    def synchronize(device=None):
        pass

    @staticmethod
    def current_stream(device=None):
        return None


class _Torch:
    cuda = _Cuda


class _Arena:
    def __init__(self):
        self.copies = 0

    def copy_(self, src):
        self.copies += 1


class _Level:
    def __init__(self, tun):
        self.t = dict(tun, use_graph=1, order=1)

    def get_tuning(self):
        return dict(self.t)

    def set_tuning(self, **t):
        if t["kernel"] == 2 and t["tile_j"] not in (4, 8):
            raise ValueError("refused")
        self.t.update(t)


class _Solver:
    stream = None
    device = "cpu"
    q = object()

    def __init__(self):
        self.arenas = []

    def new_arena(self):
        a = _Arena()
        self.arenas.append(a)
        return a


class _MG:
    """Cycle cost: a per-level table of milliseconds by (kernel, tile_j, tile_k)."""
    torch = _Torch

    def __init__(self, costs):
        self.costs = costs
        self.solver = _Solver()
        self.levels = [_Level({"kernel": 2, "tile_j": 8, "tile_k": 8}), _Level({"kernel": 0, "tile_j": 4, "tile_k": 1})]
        self.arenas_used = []

    def cycles(self, n, hist=True, arena=None):
        self.arenas_used.append(arena)
        ms = 0.0
        for lv, cost in zip(self.levels, self.costs):
            t = lv.t
            ms += cost.get((t["kernel"], t["tile_j"], t["tile_k"]), 1.0)
        _Clock.now += n * ms


def test_picks_the_fastest_candidate_per_level_and_skips_refused_ones():
    costs = [{(2, 8, 8): 0.6, (0, 4, 4): 0.5, (2, 2, 4): 0.1},       # (2, 2, 4) is refused
             {(0, 4, 1): 0.3, (0, 2, 2): 0.2}]
    mg = _MG(costs)
    res = autotune_multigrid(mg, candidates=[(0, 4, 4), (2, 2, 4), (0, 2, 2), (0, 4, 1)], cycles=4)
    got = [(t["kernel"], t["tile_j"], t["tile_k"]) for t in res["tunings"]]
    assert got == [(0, 4, 4), (0, 2, 2)]
    assert [lv.get_tuning() for lv in mg.levels] == res["tunings"]
    assert abs(res["ms_per_cycle"] - 0.7) < 1e-12
    assert all(t["use_graph"] == 1 and t["order"] == 1 for t in res["tunings"])
    assert not any((r["kernel"], r["tile_j"]) == (2, 2) for r in res["table"])


def test_times_on_a_scratch_arena_only():
    mg = _MG([{}, {}])
    autotune_multigrid(mg, candidates=[(0, 4, 4)], cycles=2)
    scratch = mg.solver.arenas
    assert len(scratch) == 1 and scratch[0].copies > 0
    assert mg.arenas_used and all(a is scratch[0] for a in mg.arenas_used)


def test_keeps_the_current_tuning_when_nothing_is_faster():
    mg = _MG([{(2, 8, 8): 0.1}, {(0, 4, 1): 0.1}])
    res = autotune_multigrid(mg, candidates=[(0, 4, 4), (0, 2, 2)], cycles=3)
    got = [(t["kernel"], t["tile_j"], t["tile_k"]) for t in res["tunings"]]
    assert got == [(2, 8, 8), (0, 4, 1)]
