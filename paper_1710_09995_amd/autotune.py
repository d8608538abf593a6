"""Tile-shape autotuner for the stage kernel.

Times candidate tunings (kernel, tile_j, tile_k) on the solver's real block
set, using a scratch copy of the state so the solver's own state is left
untouched, and keeps the fastest.  Every tuning gives bitwise identical
results (the face fluxes are the same bits whichever tile computes them), so
tuning changes speed only; ``verify=True`` re-checks that on one step.

The winner is cached in a JSON file keyed by the GPU architecture, the flow
variant and the block dimensions (``CFD_TUNE_CACHE`` overrides the path).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Tuple

DEFAULT_CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = tuple(
    (0, tj, tk, order) for order in (0, 1) for tj in (2, 4, 8) for tk in (4, 8, 16, 32, 64)) + tuple(
    (2, 8, tk, order) for order in (0, 1) for tk in (4, 8, 16, 32, 64))


def cache_path() -> str:
    p = os.environ.get("CFD_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "cfd_mi355x_tune.json")


def signature(solver) -> str:
    torch = solver.torch
    arch = torch.cuda.get_device_properties(solver.device).gcnArchName if torch.cuda.is_available() else "cpu"
    p = solver.case.params
    dims = ",".join(f"{a}x{b}x{c}" for a, b, c in solver.dims)
    raw = f"{arch}|visc{p.viscous}|fp32{p.flux_fp32}|ldt{p.local_dt}|{dims}"
    return hashlib.sha256(raw.encode()).hexdigest()[:24]


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: Dict[str, dict]) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a read-only cache location only costs a re-tune


def _time_steps(solver, arena, steps: int) -> float:
    torch = solver.torch
    stream = solver.stream if solver.stream is not None else torch.cuda.current_stream(solver.device)
    solver.step(1, hist=False, arena=arena)           # capture + warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps, hist=False, arena=arena)
    e1.record(stream)
    torch.cuda.synchronize(solver.device)
    return e0.elapsed_time(e1) / steps


def autotune(solver, candidates: Optional[Iterable[Tuple[int, int, int]]] = None, steps: int = 3,
             use_cache: bool = True, verify: bool = False, log=None) -> dict:
    """Pick and apply the fastest tuning; returns {"tuning", "ms_per_step", "table", "cached"}."""
    key = signature(solver)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        t = db[key]["tuning"]
        solver.set_tuning(**t)
        return {"tuning": t, "ms_per_step": db[key]["ms_per_step"], "table": db[key].get("table", []),
                "cached": True}
    torch = solver.torch
    scratch = solver.new_arena()
    table = []
    best = None
    for cand in (candidates or DEFAULT_CANDIDATES):
        kernel, tj, tk = cand[:3]
        order = cand[3] if len(cand) > 3 else 0
        t = {"kernel": kernel, "tile_j": tj, "tile_k": tk, "use_graph": 1, "order": order}
        try:
            solver.set_tuning(**t)
        except Exception:
            continue
        scratch.copy_(solver.q)
        ms = _time_steps(solver, scratch, steps)
        table.append(dict(t, ms_per_step=ms))
        if log:
            log(f"# tune {t}: {ms:.3f} ms/step")
        if best is None or ms < best[1]:
            best = (t, ms)
    if best is None:
        raise RuntimeError("no tuning candidate could be applied")
    if verify:
        ref = solver.get_tuning()
        outs = []
        for t in (best[0], {"kernel": 1, "tile_j": 4, "tile_k": 8, "use_graph": 0, "order": 0}):
            solver.set_tuning(**t)
            scratch.copy_(solver.q)
            solver.step(1, hist=False, arena=scratch)
            torch.cuda.synchronize(solver.device)
            outs.append([v.clone() for v in solver.interior_views(scratch)])
        for a, b in zip(*outs):
            if not torch.equal(a, b):
                raise RuntimeError("tuning changed results: bitwise check failed")
        del ref
    solver.set_tuning(**best[0])
    del scratch
    if use_cache:
        db = _load()
        db[key] = {"tuning": best[0], "ms_per_step": best[1], "table": table}
        _store(db)
    return {"tuning": best[0], "ms_per_step": best[1], "table": table, "cached": False}


MG_CANDIDATES: Tuple[Tuple[int, int, int], ...] = (
    (2, 8, 8), (2, 8, 16), (2, 4, 4), (2, 8, 4), (0, 4, 4), (0, 4, 2), (0, 4, 1), (0, 8, 4), (0, 2, 2))


def autotune_multigrid(mg, candidates: Optional[Iterable[Tuple[int, int, int]]] = None, cycles: int = 100,
                       log=None) -> dict:
    """Pick each level's tuning for the V-cycle of a Multigrid ``mg`` by
    timing whole cycles on a scratch copy of the finest state (the coarse
    levels' states are rebuilt from it in every cycle, so the solver's state
    is left untouched).  One level at a time from the finest, the others held
    at their current tunings; a candidate a level refuses is skipped.  Every
    tuning gives bitwise the same cycle, so this changes speed only.  Returns
    {"tunings" (per level), "ms_per_cycle", "table"}."""
    torch = mg.torch
    s = mg.solver
    stream = s.stream if s.stream is not None else torch.cuda.current_stream(s.device)
    scratch = s.new_arena()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def time_cycles() -> float:
        scratch.copy_(s.q)
        mg.cycles(2, hist=False, arena=scratch)       # capture + warm
        e0.record(stream)
        mg.cycles(cycles, hist=False, arena=scratch)
        e1.record(stream)
        torch.cuda.synchronize(s.device)
        return e0.elapsed_time(e1) / cycles

    table = []
    best_ms = None
    for level, lv in enumerate(mg.levels):
        cur = lv.get_tuning()
        best = (cur, time_cycles())
        table.append(dict(cur, level=level, ms_per_cycle=best[1]))
        for cand in (candidates or MG_CANDIDATES):
            kernel, tj, tk = cand[:3]
            t = {"kernel": kernel, "tile_j": tj, "tile_k": tk, "use_graph": cur["use_graph"], "order": cur["order"]}
            if all(t[k] == cur[k] for k in t):
                continue
            try:
                lv.set_tuning(**t)
            except Exception:
                continue
            ms = time_cycles()
            table.append(dict(t, level=level, ms_per_cycle=ms))
            if log:
                log(f"# tune level {level} {t}: {ms:.4f} ms/cycle")
            if ms < best[1]:
                best = (t, ms)
        lv.set_tuning(**best[0])
        best_ms = best[1]
    del scratch
    return {"tunings": [lv.get_tuning() for lv in mg.levels], "ms_per_cycle": best_ms, "table": table}
