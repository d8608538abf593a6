"""Learned warm start for steady channel-bump flows.

Pipeline (every numerical step runs in libcfd's kernels; this module only
sequences the calls and moves tensors):
  1. data:   a batch of coarse cases (one block each, own inflow Mach and bump
             height) marched to a steady state with local time stepping;
             features and primitive-deviation targets of every cell;
  2. train:  minibatch Adam on the MLP (BF16 MFMA forward, FP32 backward);
  3. start:  on a new (finer) case, the network's prediction at every cell
             becomes the initial state instead of the uniform stream;
  4. compare: steps and wall seconds until the density residual L2(R_rho)
             falls below 1e-8 of the cold start's initial residual (one
             absolute threshold for both starts; a start's own lower initial
             residual earns it nothing).
The channel cases use the steady limiter constant (cases.STEADY_LIMITER_EPS),
with which every case of the family converges linearly under local RK3
steps, so the training data are converged solutions and both starts reach
the target.  The march's tail decays at one rate whatever the start, so what
a start saves at 1e-8 is set by how little of the slowest mode it carries;
the network's own fitting error excites that mode, hence the long training
(20000 Adam iterations bring the fit's mean squared error to about 1e-6,
where 1500 left 4e-5 and a warm start slower than the cold one at 1e-8).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import cases
from .binding import Mlp, Multigrid, Solver

NET = dict(d_in=5, d_hidden=128, n_hidden=4, d_out=5)


# The steady march: multigrid V-cycles (3 levels, one RK3 step per level on
# the way down, two on the coarsest; cfd_mg_cycles) by default, plain RK3
# steps with levels = 1.  Plain RK3 at CFL 1 needs about the square of the
# cell count along the channel in steps per residual decade: on 192 x 96 x 96
# neither start reaches 1e-3 within 2e5 steps, while the cycles reach 1e-8
# in a few thousand.  Deeper hierarchies or more steps per level were
# measured to stall on transonic cases.
LEVELS, PRE, COARSE = 3, 1, 2


def _marcher(solver: Solver, levels: int):
    """A function n -> history [n, 12] advancing the solver's state by n
    steps (levels = 1) or n V-cycles."""
    if levels <= 1:
        return lambda n: solver.step(n, hist=True), None
    mg = Multigrid(solver, levels, PRE, COARSE)
    return mg.cycles, mg


def march(solver: Solver, threshold: float, max_steps: int, chunk: int = 500, log=None, levels: int = LEVELS):
    """Advance until L2(R_rho) < threshold (checked every `chunk` steps or
    cycles).

    Returns (steps, seconds, history of (step, L2(R_rho))).  The residual of
    step n is the one of the state at its start, so the count is the number
    of steps taken before a state with residual below threshold was seen.
    """
    torch = solver.torch
    adv, mg = _marcher(solver, levels)
    torch.cuda.synchronize(solver.device)
    t0 = time.perf_counter()
    done = 0
    hist = []
    while done < max_steps:
        n = min(chunk, max_steps - done)
        h = adv(n)
        r = h[:, 1].cpu().numpy()          # L2(R_rho) per step (synchronises)
        below = np.nonzero(r < threshold)[0]
        hist.extend((done + k, float(r[k])) for k in range(0, n, max(1, n // 10)))
        if below.size:
            done += int(below[0])
            break
        done += n
        if log:
            log(f"#   step {done}: L2(R_rho) = {r[-1]:.3e}")
        if not np.isfinite(r[-1]):
            break
    torch.cuda.synchronize(solver.device)
    secs = time.perf_counter() - t0
    if mg is not None:
        mg.close()
    return done, secs, hist


@dataclass
class TrainingData:
    x: object
    t: object
    conds: np.ndarray
    steps: int
    seconds: float
    final_residual: float
    info: dict = field(default_factory=dict)


def generate(n_cases: int = 256, seed: int = 0, dims=(48, 24, 24), drop: float = 1e-8, max_steps: int = 20000,
             log=None, levels: int = LEVELS) -> TrainingData:
    conds = cases.channel_conditions(n_cases, seed)
    case = cases.channel_batch_case(conds, *dims)
    s = Solver(case)
    r0 = s.step(1, hist=True)[0, 1].item()
    s.set_state(case.q0)
    steps, secs, hist = march(s, drop * r0, max_steps, log=log, levels=levels)
    x = s.mlp_features(conds)
    t = s.mlp_targets(conds)
    final = hist[-1][1] if hist else r0
    s.close()
    return TrainingData(x, t, conds, steps + 1, secs, final, {"r0": r0})


def train(data: TrainingData, iters: int = 20000, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
          log=None) -> Mlp:
    import torch
    net = Mlp(cases.mlp_init(**NET, seed=seed), **NET)
    n = data.x.shape[0]
    gen = torch.Generator(device=net.device).manual_seed(seed)
    for it in range(iters):
        idx = torch.randint(0, n, (batch,), device=net.device, generator=gen, dtype=torch.int32)
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / iters))     # cosine decay
        loss = net.train_step(data.x, data.t, idx, lr=rate)
        if log and (it % 500 == 0 or it == iters - 1):
            log(f"#   train it {it}: loss {loss.item():.3e}")
    return net


def warm_state(solver: Solver, net: Mlp, conds):
    """Write the network's prediction into the solver's state (interior cells)."""
    x = solver.mlp_features(conds)
    y = net.forward(x)
    solver.mlp_to_state(y, conds)


DECADES = tuple(10.0 ** -e for e in range(1, 9))     # residual drops 1e-1 .. 1e-8


def march_decades(solver: Solver, r_ref: float, max_steps: int, chunk: int = 250, t_extra: float = 0.0,
                  log=None, log_every: int = 20000, advance=None):
    """March up to max_steps (steps, or cycles with a multigrid `advance`);
    for every drop d in DECADES record the first step (and the wall seconds,
    plus t_extra) at which L2(R_rho) < d * r_ref."""
    torch = solver.torch
    advance = advance or (lambda n: solver.step(n, hist=True))
    torch.cuda.synchronize(solver.device)
    t0 = time.perf_counter()
    reached = {}
    done = 0
    last = float("nan")
    while done < max_steps and len(reached) < len(DECADES):
        n = min(chunk, max_steps - done)
        r = advance(n)[:, 1].cpu().numpy()
        now = time.perf_counter() - t0 + t_extra
        for d in DECADES:
            if d in reached:
                continue
            hit = np.nonzero(r < d * r_ref)[0]
            if hit.size:
                reached[d] = (done + int(hit[0]), now)
        if log and (done + n) // log_every > done // log_every:
            log(f"#   step {done + n}: drop {r[-1] / r_ref:.2e}, {now:.1f} s")
        done += n
        last = float(r[-1])
        if not np.isfinite(last):
            break
    return reached, done, last


@dataclass
class Comparison:
    mach: float
    hb: float
    r_cold0: float
    r_warm0: float
    cold: dict          # drop -> (steps, seconds)
    warm: dict
    cold_final: float
    warm_final: float
    steps_cap: int
    inference_s: float


def compare(net: Mlp, conds, dims=(192, 96, 96), max_steps: int = 20000, log=None, chunk: int = 250,
            levels: int = LEVELS) -> List[Comparison]:
    """Cold (uniform stream) vs warm (network) start on each condition; one
    absolute reference, the cold start's initial residual, for both; the same
    steady march (multigrid cycles, or RK3 steps with levels = 1) for both."""
    out = []
    for mach, hb in conds:
        case = cases.channel_case(*dims, mach=float(mach), hb=float(hb))
        s = Solver(case)
        adv, mg = _marcher(s, levels)
        r_cold0 = s.step(1, hist=True)[0, 1].item()     # residual of the uniform stream
        s.set_state(case.q0)
        cold, _, cold_final = march_decades(s, r_cold0, max_steps, chunk, log=log, advance=adv)
        s.set_state(case.q0)
        s.torch.cuda.synchronize(s.device)
        t0 = time.perf_counter()
        warm_state(s, net, [(mach, hb)])
        s.torch.cuda.synchronize(s.device)
        t_inf = time.perf_counter() - t0
        r_warm0 = s.step(1, hist=True)[0, 1].item()
        warm_state(s, net, [(mach, hb)])
        warm, _, warm_final = march_decades(s, r_cold0, max_steps, chunk, t_extra=t_inf, log=log, advance=adv)
        c = Comparison(float(mach), float(hb), r_cold0, r_warm0, cold, warm, cold_final, warm_final, max_steps,
                       t_inf)
        if log:
            log(f"# M={mach:.3f} h={hb:.3f}: r0 cold {r_cold0:.3e} warm {r_warm0:.3e}; "
                f"cold {summarise(cold)}; warm {summarise(warm)}")
        out.append(c)
        if mg is not None:
            mg.close()
        s.close()
    return out


def summarise(reached: dict) -> str:
    return ", ".join(f"{d:.0e}:{v[0]}st/{v[1]:.2f}s" for d, v in sorted(reached.items(), reverse=True))


def deepest_common(c: Comparison) -> Optional[float]:
    common = [d for d in DECADES if d in c.cold and d in c.warm]
    return min(common) if common else None


TARGET = DECADES[-1]


def target_seconds(res: List[Comparison]):
    """Per case (cold s, warm s) to the 1e-8 target; a start that did not reach
    it within the cap counts as None."""
    out = []
    for c in res:
        out.append((c.cold[TARGET][1] if TARGET in c.cold else None,
                    c.warm[TARGET][1] if TARGET in c.warm else None))
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned warm start: data, training, cold vs warm comparison")
    ap.add_argument("--cases", type=int, default=256)
    ap.add_argument("--coarse", type=int, nargs=3, default=[48, 24, 24])
    ap.add_argument("--fine", type=int, nargs=3, default=[192, 96, 96])
    ap.add_argument("--data-steps", type=int, default=20000, help="cap on the training data's steps or cycles")
    ap.add_argument("--levels", type=int, default=LEVELS, help="multigrid levels of the steady march (1: plain RK3)")
    ap.add_argument("--iters", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--test", type=int, default=4)
    ap.add_argument("--test-seed", type=int, default=12345)
    ap.add_argument("--cap", type=int, default=20000, help="steps (levels 1) or cycles per start")
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--test-skip", type=int, default=0, help="skip the first K held-out conditions")
    ap.add_argument("--save-net", default=None, help="write the trained weights (.npz)")
    ap.add_argument("--load-net", default=None, help="skip data and training; use these weights (.npz)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)   # noqa: E731
    t0 = time.perf_counter()
    if a.load_net:
        with np.load(a.load_net, allow_pickle=False) as z:
            net = Mlp([(z[f"w{k}"], z[f"b{k}"]) for k in range(len(z.files) // 2)], **NET)
        data = None
        t1 = t2 = time.perf_counter()
    else:
        data = generate(a.cases, 0, tuple(a.coarse), drop=1e-8, max_steps=a.data_steps, log=log, levels=a.levels)
        log(f"# data: {data.x.shape[0]} points from {a.cases} cases, {data.steps} steps in {data.seconds:.1f} s, "
            f"residual {data.info['r0']:.3e} -> {data.final_residual:.3e}")
        t1 = time.perf_counter()
        net = train(data, iters=a.iters, batch=a.batch, log=log)
        net.torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"# training: {a.iters} iterations in {t2 - t1:.1f} s")
        if a.save_net:
            flat = {}
            for k, (w, b) in enumerate(net.params()):
                flat[f"w{k}"], flat[f"b{k}"] = w, b
            np.savez(a.save_net, **flat)
    tests = cases.channel_conditions(a.test_skip + a.test, a.test_seed)[a.test_skip:]
    res = compare(net, tests, tuple(a.fine), a.cap, log=log, chunk=a.chunk, levels=a.levels)
    summary = []
    for c in res:
        d = deepest_common(c)
        summary.append({"mach": c.mach, "hb": c.hb, "r_cold0": c.r_cold0, "r_warm0": c.r_warm0,
                        "cold": {f"{k:.0e}": v for k, v in c.cold.items()},
                        "warm": {f"{k:.0e}": v for k, v in c.warm.items()},
                        "cold_final_drop": c.cold_final / c.r_cold0, "warm_final_drop": c.warm_final / c.r_cold0,
                        "deepest_common_drop": d,
                        "speedup_steps": (c.cold[d][0] / max(1, c.warm[d][0])) if d else None,
                        "speedup_seconds": (c.cold[d][1] / max(1e-9, c.warm[d][1])) if d else None,
                        "inference_s": c.inference_s, "cap": c.steps_cap,
                        "target_cold": c.cold.get(TARGET), "target_warm": c.warm.get(TARGET)})
    ts = target_seconds(res)
    both = [(x, y) for x, y in ts if x is not None and y is not None]
    out = {"train_cases": a.cases, "coarse": a.coarse, "fine": a.fine, "levels": a.levels,
           "data_steps": data.steps if data else None, "data_seconds": data.seconds if data else None,
           "train_iters": a.iters, "train_seconds": t2 - t1, "net": a.load_net or "trained here",
           "data_final_drop": data.final_residual / data.info["r0"] if data else None,
           "total_seconds": time.perf_counter() - t0, "tests": summary,
           "target": TARGET, "reached_cold": sum(x is not None for x, _ in ts),
           "reached_warm": sum(y is not None for _, y in ts),
           "median_seconds_cold": float(np.median([x for x, _ in both])) if both else None,
           "median_seconds_warm": float(np.median([y for _, y in both])) if both else None}
    print(json.dumps(out), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
