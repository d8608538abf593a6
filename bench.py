#!/usr/bin/env python3
"""Benchmark of the hot path: full SSP-RK3 time steps (ghost fill, time step,
three residual + stage updates, norms) on one MI355X.

Default workload: one GPU's share at the paper's scale, 16 curvilinear
blocks of 512 x 512 x 144 cells (604 M cells) joined face to face,
compressible Navier-Stokes over a wall bump, FP64 arithmetic, seeded
pressure pulses (synthetic inputs generated on the device).  Prints one JSON
line with the cell-stage update rate, the stage kernel's roofline figures,
the FP32-flux variant's error against FP64 and the CPU oracle's rate on a
bounded sample.

Timing (the paper's protocol: best of 5 runs): W untimed warm-up steps,
then 5 runs of exactly K steps, each bracketed by device synchronisation and
HIP events on the solver's stream (graph replay, the production path);
`value` is the best run, the median is reported beside it.  A further pass
of K steps with the library's kernel profiling on (eager launches, a
hipEvent pair around every stage-kernel launch on its stream) gives the
stage kernel's mean duration for the roofline entry.  Then the state is
reset to the initial field and K steps are run again, and a second context
with FP32 fluxes runs the same K steps from the same field: the relative L2
of its state against the FP64 one is reported (and its own best rate).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK = 78.6   # TFLOP/s


def stage_bytes_per_cell(local_dt: bool) -> float:
    """Algorithmic HBM bytes per interior cell per stage-kernel launch, averaged
    over the three stages: stencil state 40 B (read once), metrics 80 B
    (S_i, S_j, S_k, V), write 40 B; stages 2-3 also read Q^n pointwise (40 B);
    local time stepping reads one more double per cell."""
    s1 = 40 + 80 + 40
    s23 = s1 + 40
    extra = 8 if local_dt else 0
    return (s1 + 2 * s23) / 3.0 + extra


def make_case(name: str, flux: str, device=None):
    from paper_1710_09995_amd import cases
    fp32 = 1 if flux == "fp32" else 0
    if name == "bump_ns":
        c = cases.bump_ns_case(256, 128, 128, seed=0)
        label = "bump_ns_256x128x128"
    elif name == "vortex":
        c = cases.vortex_case(32, seed=0)
        label = "euler_vortex_32^3"
    elif name == "batched":
        c = cases.batched_euler_case(64, seed=0)
        label = "batched_euler_64blk"
    elif name == "paper_share":
        c = cases.paper_share_case(seed=0, flux_fp32=fp32, device=device,
                                   log=lambda m: print(m, file=sys.stderr, flush=True))
        label = "ns_16x512x512x144"
    else:
        raise SystemExit(f"unknown workload {name}")
    return c.with_params(flux_fp32=fp32), label


def cpu_baseline(name: str, flux: str, budget_s: float = 12.0):
    """The oracle as it stands, on a bounded sample of the same workload."""
    import numpy as np  # noqa: F401
    from oracle import solver as osol
    from paper_1710_09995_amd import cases
    if name == "paper_share":
        c = cases.paper_share_case(nbx=1, nbz=1, ni=64, nj=64, nk=18, seed=0, flux_fp32=0)
        sample = ("one 64x64x18 block of the same flow, grid family and boundaries (wall bump, tanh "
                  "stretching, pulses, periodic in x and z), FP64 oracle RK3 steps")
    elif name == "bump_ns":
        c = cases.bump_ns_case(64, 32, 32, seed=0)
        sample = "bump_ns 64x32x32 sub-block (same flow, grid family and BCs), FP64 oracle RK3 steps"
    elif name == "vortex":
        c = cases.vortex_case(32, seed=0)
        sample = "euler vortex 32^3, FP64 oracle RK3 steps"
    else:
        c = cases.batched_euler_case(8, seed=0, lo=16, hi=40, flux_fp32=0)
        sample = "batched euler 8 blocks dims in [16,40), FP64 oracle RK3 steps"
    st = osol.setup(c)
    t0 = time.perf_counter()
    n = 0
    while True:
        osol.step(st)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    rate = c.ncells * 3 * n / dt / 1e6
    return {"value": rate, "unit": "Mcell-stage/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}; {n} steps of {c.ncells} cells in {dt:.1f} s, single-threaded NumPy"}


STAGE_SOURCES = ("kernels_ring.hip", "stage_common.hpp", "physics.hpp", "cfd_internal.hpp")
HIGHORDER_SOURCES = ("kernels_highorder.hip", "physics.hpp")


def read_profile_value(kernel_label: str, kind: str, key: str, sources=STAGE_SOURCES):
    """A per-launch figure from a committed rocprofv3 --pmc summary
    (profiles/<label>_<kind>.txt), valid only while the sources of the
    kernels it measured are unchanged."""
    path = os.path.join(ROOT, "profiles", f"{kernel_label}_{kind}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha") != source_sha(sources):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def read_traffic(kernel_label: str):
    """HBM bytes per stage launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return read_profile_value(kernel_label, "pmc", "hbm_bytes_per_launch")


def source_sha(sources=STAGE_SOURCES) -> str:
    """Hash of the sources that define the measured kernels (by default the
    plane-ring stage kernel, which the headline's counter summaries measure)."""
    h = hashlib.sha256()
    for f in sources:
        p = os.path.join(ROOT, "paper_1710_09995_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def timed_steps(torch, s, steps: int, stream) -> float:
    """Milliseconds of `steps` RK3 steps between two synchronised HIP events on `stream`."""
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, hist=False)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def rel_l2_interior(torch, s, arena, ref_host) -> float:
    """Relative L2 over all interior cells and components of the state arena
    `arena` of solver s against a reference arena of the same layout held in
    host memory (uploaded block by block), summed on the device in FP64."""
    num = torch.zeros((), dtype=torch.float64, device=arena.device)
    den = torch.zeros((), dtype=torch.float64, device=arena.device)
    for va, vh in zip(s.interior_views(arena), s.interior_views(ref_host)):
        vb = vh.to(arena.device)
        num += torch.sum((va - vb) ** 2)
        den += torch.sum(vb * vb)
        del vb
    return float(torch.sqrt(num / den))


def fp32_flux_check(torch, s, case, a, stream, remake) -> dict:
    """The FP32-flux / FP64-state variant against the FP64 path: both run K
    steps from the initial field; the relative L2 of the FP32-flux state
    against the FP64 state (itself pinned to the oracle at 1e-12 per step),
    and the FP32-flux variant's own best rate (best of two runs).  The FP64
    state waits in host memory and the FP64 context, its workspace and the
    device-generated inputs are released first (the one-GPU share needs
    about 250 GB of HBM per context); remake() rebuilds the inputs."""
    from paper_1710_09995_amd.binding import Solver
    s.set_state(case.q0)
    s.step(a.steps, hist=False)
    torch.cuda.synchronize()
    ref_host = s.q.cpu()
    s.close()
    s.q = None
    s.workspace = None
    case.nodes.clear()
    torch.cuda.empty_cache()
    case32 = remake()
    s32 = Solver(case32, device="cuda:0")
    case32.nodes.clear()
    torch.cuda.empty_cache()
    s32.step(a.steps, hist=False)
    torch.cuda.synchronize()
    err = rel_l2_interior(torch, s32, s32.q, ref_host)
    del ref_host
    s32.step(a.warmup, hist=False)
    reps = [timed_steps(torch, s32, a.steps, stream) for _ in range(min(2, max(1, a.reps)))]
    ms = min(reps)
    s32.close()
    del s32
    torch.cuda.empty_cache()
    rate = case.ncells * 3 * a.steps / (ms / 1e3) / 1e6
    print(f"# FP32-flux / FP64-state after {a.steps} steps from the same field: relative L2 against the FP64 "
          f"state {err:.3e}; its best rate {rate:.1f} Mcell-stage/s", file=sys.stderr, flush=True)
    return {"steps": a.steps, "rel_l2_vs_fp64": err, "gate": 1e-5, "value": round(rate, 2),
            "unit": "Mcell-stage/s", "ms_per_step": round(ms / a.steps, 4)}


def bench_op(a) -> int:
    """One high-order operator alone: K launches per direction after W
    warm-up launches, hipEvents on the launch stream; algorithmic bytes = the
    input field read once + the outputs written once."""
    import torch
    from paper_1710_09995_amd.binding import staggered_diff6, wcns5_edges
    n, nvar, h = (256, 128, 128), 5, 1.0 / 256
    cells = n[0] * n[1] * n[2]
    pad = 5 if a.op == "diff6" else 10
    stream = torch.cuda.current_stream()
    per_dir = {}
    for d in range(3):
        shape = [nvar, n[2], n[1], n[0]]
        shape[3 - d] += pad
        g = torch.Generator(device="cuda").manual_seed(d)
        f = torch.rand(shape, dtype=torch.float64, device="cuda", generator=g)
        if a.op == "diff6":
            out = torch.empty((nvar, n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
            run = lambda: staggered_diff6(f, n, d, h, out=out)   # noqa: E731
            out_elems = out.numel()
        else:
            run = lambda: wcns5_edges(f, n, d)                   # noqa: E731
            out_elems = 2 * run()[0].numel()
        for _ in range(a.warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        nbytes = 8 * (f.numel() + out_elems)
        per_dir["ijk"[d]] = {"ms": round(ms, 5), "bytes": nbytes, "GB_s": round(nbytes / (ms / 1e3) / 1e9, 1)}
    # a plain device copy of the same bytes, for the achievable-bandwidth context
    src = torch.rand(int(per_dir["k"]["bytes"] // 16), dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 16 * src.numel() / (e0.elapsed_time(e1) / a.steps / 1e3) / 1e9
    ms = sum(v["ms"] for v in per_dir.values()) / 3
    nbytes = sum(v["bytes"] for v in per_dir.values()) / 3
    achieved = nbytes / (ms / 1e3) / 1e9
    print(json.dumps({
        "metric": ("Mcell/s of the Eq. (2) sixth-order staggered difference" if a.op == "diff6" else
                   "Mcell/s of the WCNS-E-5 cell-edge interpolation (left and right states)") +
                  " (5 variables, mean over i, j, k)",
        "value": round(cells / (ms / 1e3) / 1e6, 1), "unit": "Mcell/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform face fields)",
        "config": {"workload": ("staggered_diff6" if a.op == "diff6" else "wcns5_edges") + "_256x128x128x5",
                   "per_direction": per_dir,
                   "plain_copy_GB_s": round(copy_gbs, 1), "frac_of_plain_copy": round(achieved / copy_gbs, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_window6_i / k_window6_march<" + ("Eq2Op" if a.op == "diff6" else "Wcns5Op") + ">",
                     "mean_launch_ms": round(ms, 5),
                     "algorithmic_bytes_per_launch": nbytes},
        "cpu_baseline": None}), flush=True)
    return 0


def bench_wcns5_euler(a) -> int:
    """The periodic inviscid WCNS-E-5 residual of a 256x128x128 block (a
    smooth seeded flow): K residuals after W warm-up ones, hipEvents on the
    launch stream.  The roofline counts each kernel of the pipeline reading
    its inputs once and writing its outputs once (padding, the face states
    with Roe's flux in one pass, Eq. 2 with the running sum), i.e. the
    intermediates' HBM traffic."""
    import numpy as np
    import torch
    from paper_1710_09995_amd.binding import (c4_viscous_add_curv_periodic, c4_viscous_add_periodic,
                                              wcns5_euler_residual_curv_periodic, wcns5_euler_residual_periodic,
                                              wcns5_metrics_periodic)
    viscous = a.op in ("ns_periodic", "ns_curv")
    curv = a.op in ("wcns5_curv", "ns_curv")
    n = (256, 128, 128)
    ni, nj, nk = n
    cells = ni * nj * nk
    rng = np.random.default_rng(0)
    ph = rng.uniform(0, 2 * np.pi, 4)
    z, y, x = np.meshgrid(np.arange(nk) / nk, np.arange(nj) / nj, np.arange(ni) / ni, indexing="ij")
    s2 = 2 * np.pi
    rho = 1 + 0.2 * np.sin(s2 * x + ph[0]) * np.cos(s2 * y + ph[1]) + 0.1 * np.sin(s2 * z + ph[2])
    u, v, w = 0.5 + 0.1 * np.sin(s2 * y + ph[3]), 0.1 * np.sin(s2 * z), 0.1 * np.sin(s2 * x)
    p = 1 + 0.1 * np.cos(s2 * (x + y + z))
    q = torch.from_numpy(np.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)])).cuda()
    h = (1.0 / ni, 1.0 / nj, 1.0 / nk)
    out = torch.empty_like(q)
    work = None
    from paper_1710_09995_amd import binding as B
    import ctypes as C
    nb = C.c_size_t()
    B._check(B.lib().cfd_wcns5_euler_work_bytes((C.c_int32 * 3)(ni, nj, nk), C.byref(nb)))
    work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    vwork = None
    if viscous:
        B._check((B.lib().cfd_c4_viscous_curv_work_bytes if curv else B.lib().cfd_c4_viscous_work_bytes)(
            (C.c_int32 * 3)(ni, nj, nk), C.byref(nb)))
        vwork = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    setup_ms = None
    if curv:   # a wavy periodic grid on the box 1 x 1/2 x 1/2: each coordinate displaced by sines of the others
        L, amp = (1.0, 0.5, 0.5), 0.05
        zb, yb, xb = np.meshgrid((np.arange(nk) + 0.5) * L[2] / nk, (np.arange(nj) + 0.5) * L[1] / nj,
                                 (np.arange(ni) + 0.5) * L[0] / ni, indexing="ij")
        wx, wy, wz = s2 * xb / L[0], s2 * yb / L[1], s2 * zb / L[2]
        xv = torch.from_numpy(np.stack([xb + amp * L[0] * np.sin(wy) * np.sin(wz),
                                        yb + amp * L[1] * np.sin(wz) * np.sin(wx),
                                        zb + amp * L[2] * np.sin(wx) * np.sin(wy)])).cuda()
        del xb, yb, zb, wx, wy, wz
        S, jinv = wcns5_metrics_periodic(xv, np.diag(L))
        torch.cuda.synchronize()
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m0.record(torch.cuda.current_stream())
        S, jinv = wcns5_metrics_periodic(xv, np.diag(L))
        m1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        setup_ms = m0.elapsed_time(m1)

    def residual():
        if curv:
            wcns5_euler_residual_curv_periodic(q, S, jinv, out=out, work=work)
        else:
            wcns5_euler_residual_periodic(q, h, out=out, work=work)
        if viscous and curv:
            c4_viscous_add_curv_periodic(q, out, S, jinv, 1.4, 0.72, 1e-3, 110.4 / 288.15, work=vwork)
        elif viscous:
            c4_viscous_add_periodic(q, out, h, 1.4, 0.72, 1e-3, 110.4 / 288.15, work=vwork)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        residual()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        residual()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    # Algorithmic bytes of the passes this block runs (each reading its inputs and writing its outputs once):
    # inviscid, per direction, the state (5 in) and the face area vectors (3, curvilinear), R written along i and
    # read and written along j and k, J^{-1} read by the last pass.
    nbytes = 8 * cells * (3 * 5 + (5 + 2 * 5 + 2 * 5))
    if curv:
        nbytes += 8 * cells * (3 * 3 + 1)
    if viscous and curv:   # phi with the i derivatives (Q in; 4 + 4 out), the j and k derivatives (4 in, 4 out
        # each), the cell metrics (9 in, 9 out) and per direction the face metrics (9 + 1 in, 7 out) that this
        # one-shot call forms each time, then per direction the fused faces and differences (phi 4 + gradients 8
        # + face metrics 7 + S_d 3 + J^{-1} 1 in, r 4 in and out)
        nbytes += 8 * cells * ((5 + 8) + 2 * (4 + 4) + (9 + 9) + 3 * (10 + 7) + 3 * (4 + 8 + 7 + 3 + 1 + 4 + 4))
    elif viscous:   # phi (Q in, 4 out), gradients (4 in, 12 out), per direction faces (16 in, 4 out) and the sum
        nbytes += 8 * cells * ((5 + 4) + (4 + 12) + 3 * ((4 + 8) + 4) + 3 * (4 + 8))
    achieved = nbytes / (ms / 1e3) / 1e9
    label = ("ns_wcns5_c4" if viscous else "wcns5_euler") + ("_curv" if curv else "") + "_periodic_256x128x128"
    traffic = read_profile_value(label, "pmc", "hbm_bytes_per_residual", HIGHORDER_SOURCES)
    print(json.dumps({
        "metric": "Mcell/s of the periodic " + ("curvilinear " if curv else "") +
                  ("Navier-Stokes (WCNS-E-5 inviscid + fourth-order viscous)" if viscous else "inviscid WCNS-E-5") +
                  " residual (three directions)",
        "value": round(cells / (ms / 1e3) / 1e6, 1), "unit": "Mcell/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded smooth periodic flow)",
        "config": {"workload": ("ns_wcns5_c4" if viscous else "wcns5_euler") + ("_curv" if curv else "") +
                               "_periodic_256x128x128",
                   "metrics_setup_ms": None if setup_ms is None else round(setup_ms, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_rate_gbs": None if traffic is None else round(traffic / (ms / 1e3) / 1e9, 1),
                     "kernel": "pipeline: k_wcns5_euler_rows, k_wcns5_euler_march<1|2>"
                               + (" (the last pass dividing by J^-1)" if curv else "")
                               + (", k_c4_phi_grads_i, k_c4_grads_march<1|2>, k_c4_cell_metrics, k_c4_face_metrics, "
                                  "k_c4_visc_rows, k_c4_visc_march<1|2>" if viscous and curv else
                                  ", k_c4_phi, k_c4_grads, k_c4_visc_faces, k_c4_flux_sub" if viscous else ""),
                     "mean_ms": round(ms, 4), "pipeline_bytes": nbytes},
        "cpu_baseline": None}), flush=True)
    return 0


def bench_implicit(a) -> int:
    """Implicit steps (backward Euler, 4 point-Jacobi sweeps) of the inviscid
    WCNS-E-5 residual on the wavy periodic 256x128x128 grid of --op
    wcns5_curv, at 5 times the CFL-1 step; K steps after W warm-up ones,
    hipEvents on the launch stream.  Algorithmic bytes: the residual's
    pipeline plus, per sweep, each cell's state, update, residual, metrics,
    radii, J^{-1} and diagonal read once and the update written once."""
    import numpy as np
    import torch
    from paper_1710_09995_amd.binding import (wcns5_implicit_steps_curv_periodic, wcns5_metrics_periodic,
                                              wcns5_time_step_curv_periodic)
    n = (256, 128, 128)
    ni, nj, nk = n
    cells = ni * nj * nk
    rng = np.random.default_rng(0)
    ph = rng.uniform(0, 2 * np.pi, 4)
    s2 = 2 * np.pi
    z, y, x = np.meshgrid(np.arange(nk) / nk, np.arange(nj) / nj, np.arange(ni) / ni, indexing="ij")
    rho = 1 + 0.2 * np.sin(s2 * x + ph[0]) * np.cos(s2 * y + ph[1]) + 0.1 * np.sin(s2 * z + ph[2])
    u, v, w = 0.5 + 0.1 * np.sin(s2 * y + ph[3]), 0.1 * np.sin(s2 * z), 0.1 * np.sin(s2 * x)
    p = 1 + 0.1 * np.cos(s2 * (x + y + z))
    q0 = torch.from_numpy(np.stack([rho, rho * u, rho * v, rho * w,
                                    p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)])).cuda()
    L, amp = (1.0, 0.5, 0.5), 0.05
    zb, yb, xb = np.meshgrid((np.arange(nk) + 0.5) * L[2] / nk, (np.arange(nj) + 0.5) * L[1] / nj,
                             (np.arange(ni) + 0.5) * L[0] / ni, indexing="ij")
    wx, wy, wz = s2 * xb / L[0], s2 * yb / L[1], s2 * zb / L[2]
    xv = torch.from_numpy(np.stack([xb + amp * L[0] * np.sin(wy) * np.sin(wz),
                                    yb + amp * L[1] * np.sin(wz) * np.sin(wx),
                                    zb + amp * L[2] * np.sin(wx) * np.sin(wy)])).cuda()
    S, jinv = wcns5_metrics_periodic(xv, np.diag(L))
    dt = 5.0 * float(wcns5_time_step_curv_periodic(q0, S, jinv, 1.0).cpu()[0])
    q = q0.clone()
    sweeps = 4
    for _ in range(a.warmup):
        wcns5_implicit_steps_curv_periodic(q, S, jinv, dt, 1, sweeps)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        wcns5_implicit_steps_curv_periodic(q, S, jinv, dt, 1, sweeps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    # the residual's row and marching passes (per direction Q and the area vectors in, R written or updated,
    # J^{-1} in the last), then the implicit passes
    nbytes = 8 * cells * (3 * 5 + (5 + 2 * 5 + 2 * 5) + 3 * 3 + 1)
    nbytes += 8 * cells * ((5 + 9 + 3) + (5 + 3 + 1 + 1 + 5))           # radii; diagonal and first iterate
    nbytes += sweeps * 8 * cells * (5 + 5 + 5 + 9 + 3 + 1 + 1 + 5)      # one sweep
    nbytes += 8 * cells * 15                                            # q += dQ
    achieved = nbytes / (ms / 1e3) / 1e9
    finite = bool(torch.isfinite(q).all())
    print(json.dumps({
        "metric": "Mcell/s of implicit steps (backward Euler, 4 Jacobi sweeps) on the curvilinear WCNS-E-5 residual",
        "value": round(cells / (ms / 1e3) / 1e6, 1), "unit": "Mcell/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded smooth periodic flow, wavy grid)",
        "config": {"workload": "implicit_wcns5_curv_periodic_256x128x128", "sweeps": sweeps, "cfl": 5.0,
                   "finite": finite},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "pipeline: residual (k_wcns5_euler_rows, k_wcns5_euler_march<1|2>), k_impl_lambda, k_impl_diag, "
                               "k_impl_sweep x4, k_impl_apply",
                     "mean_ms": round(ms, 4), "pipeline_bytes": nbytes},
        "cpu_baseline": None}), flush=True)
    return 0


def bench_ns_blocks(a) -> int:
    """RK3 Navier-Stokes steps on the wavy periodic 256x128x128 grid of --op
    wcns5_curv cut into 2 x 2 x 2 blocks joined face to face, against the same
    steps on the unsplit periodic block in the same run: one call of K steps
    after one call of W warm-up steps each (a call forms the viscous face
    metrics once), hipEvents on the launch stream."""
    import numpy as np
    import torch
    from paper_1710_09995_amd.binding import (wcns5_metrics_periodic, wcns5_ns_steps_blocks,
                                              wcns5_ns_steps_curv_periodic, wcns5_time_step_curv_periodic)
    n = (256, 128, 128)
    ni, nj, nk = n
    cells = ni * nj * nk
    rng = np.random.default_rng(0)
    ph = rng.uniform(0, 2 * np.pi, 4)
    s2 = 2 * np.pi
    z, y, x = np.meshgrid(np.arange(nk) / nk, np.arange(nj) / nj, np.arange(ni) / ni, indexing="ij")
    rho = 1 + 0.2 * np.sin(s2 * x + ph[0]) * np.cos(s2 * y + ph[1]) + 0.1 * np.sin(s2 * z + ph[2])
    u, v, w = 0.5 + 0.1 * np.sin(s2 * y + ph[3]), 0.1 * np.sin(s2 * z), 0.1 * np.sin(s2 * x)
    p = 1 + 0.1 * np.cos(s2 * (x + y + z))
    q0 = torch.from_numpy(np.stack([rho, rho * u, rho * v, rho * w,
                                    p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)])).cuda()
    L, amp = (1.0, 0.5, 0.5), 0.05
    zb, yb, xb = np.meshgrid((np.arange(nk) + 0.5) * L[2] / nk, (np.arange(nj) + 0.5) * L[1] / nj,
                             (np.arange(ni) + 0.5) * L[0] / ni, indexing="ij")
    wx, wy, wz = s2 * xb / L[0], s2 * yb / L[1], s2 * zb / L[2]
    xv = torch.from_numpy(np.stack([xb + amp * L[0] * np.sin(wy) * np.sin(wz),
                                    yb + amp * L[1] * np.sin(wz) * np.sin(wx),
                                    zb + amp * L[2] * np.sin(wx) * np.sin(wy)])).cuda()
    S, jinv = wcns5_metrics_periodic(xv, np.diag(L))
    mu = 1e-3
    dt = float(wcns5_time_step_curv_periodic(q0, S, jinv, 0.5, 1.4, True, 0.72, mu).cpu()[0])
    half = (ni // 2, nj // 2, nk // 2)
    sls, nbr = [], []
    for c in range(2):
        for b in range(2):
            for aa in range(2):
                sls.append((slice(c * half[2], (c + 1) * half[2]), slice(b * half[1], (b + 1) * half[1]),
                            slice(aa * half[0], (aa + 1) * half[0])))
                idx = lambda i, j, k: (k % 2) * 4 + (j % 2) * 2 + (i % 2)          # noqa: E731
                nbr.append([idx(aa - 1, b, c), idx(aa + 1, b, c), idx(aa, b - 1, c), idx(aa, b + 1, c),
                            idx(aa, b, c - 1), idx(aa, b, c + 1)])
    qs = [q0[(slice(None),) + sl].contiguous() for sl in sls]
    Ss = [S[(slice(None), slice(None)) + sl].contiguous() for sl in sls]
    Js = [jinv[sl].contiguous() for sl in sls]
    qw = q0.clone()
    stream = torch.cuda.current_stream()

    def timed(fn):
        if a.warmup > 0:
            fn(a.warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(a.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / a.steps
    ms_blocks = timed(lambda k: wcns5_ns_steps_blocks(qs, Ss, Js, nbr, dt, k, 1.4, 0.1, 1e-6, 0.72, mu))
    ms_whole = timed(lambda k: wcns5_ns_steps_curv_periodic(qw, S, jinv, dt, k, 1.4, 0.1, 1e-6, 0.72, mu))
    finite = bool(all(torch.isfinite(t).all() for t in qs))
    print(json.dumps({
        "metric": "Mcell-stage/s of RK3 Navier-Stokes steps (WCNS-E-5 + fourth-order viscous) on 8 curvilinear "
                  "blocks joined face to face",
        "value": round(cells * 3 / (ms_blocks / 1e3) / 1e6, 1), "unit": "Mcell-stage/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_blocks, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded smooth periodic flow, "
        "wavy grid)",
        "config": {"workload": "ns_wcns5_c4_blocks_2x2x2_of_256x128x128", "blocks": 8, "finite": finite,
                   "unsplit_ms_per_step": round(ms_whole, 4),
                   "unsplit_mcell_stage_s": round(cells * 3 / (ms_whole / 1e3) / 1e6, 1)},
        "roofline": None, "cpu_baseline": None}), flush=True)
    return 0


def bench_ns_share(a) -> int:
    """RK3 Navier-Stokes steps of the paper's operator (WCNS-E-5 and the
    fourth-order viscous terms) on the one-GPU share's geometry closed by
    ghost blocks (no-slip wall below, far field above the wall-normal
    direction): 2 x 2 of its 512 x 512 x 144 blocks tiling x and z (151 M
    cells; the operator's working arrays take some 430 B per cell, so the 16
    blocks of the share do not fit with them), a uniform stream at M 0.8,
    Re 1e6 per unit length.  One call of K steps after one call of W warm-up
    steps at a fixed step (a call forms the viscous face metrics once),
    hipEvents on the launch stream."""
    import math
    import numpy as np
    import torch
    from paper_1710_09995_amd import cases
    from paper_1710_09995_amd.binding import WcnsClosedTiling
    nb, ni, nj, nk = 2, 512, 512, 144
    t0 = time.perf_counter()
    Xv, P = cases.paper_share_vertices(nb, nb, ni, nj, nk)
    xv = torch.from_numpy(Xv).cuda()
    del Xv
    N = (nb * ni, nb * nj, nk)
    cuts = {0: [b * ni for b in range(nb + 1)], 1: [b * nj for b in range(nb + 1)]}
    uinf = (0.8 * math.sqrt(1.4), 0.0, 0.0)
    tl = WcnsClosedTiling(xv, P, 2, (3, 1), uinf, 1.4, cuts=cuts)      # no-slip wall below, far field above
    del xv
    q0 = torch.from_numpy(cases.uniform_state((ni, nj, nk), cases.Params(mach=0.8))).cuda()
    qs = [q0.clone() for _ in tl.owners]
    del q0
    setup_s = time.perf_counter() - t0
    visc = (0.72, uinf[0] / 1e6, 110.4 / 288.15)
    dt = 1e-5
    work = None
    stream = torch.cuda.current_stream()
    if a.warmup > 0:
        tl.steps(qs, dt, a.warmup, viscous=visc, work=work)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tl.steps(qs, dt, a.steps, viscous=visc, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    cells = N[0] * N[1] * N[2]
    finite = bool(all(torch.isfinite(t).all() for t in qs))
    # Algorithmic bytes per cell and stage of the passes an owner block runs (each reading its inputs and writing
    # its outputs once; the ghost blocks' fill and the face metrics, formed once per call, left out): inviscid,
    # per direction Q (5) and S_d (3) in, R written along i and updated along j and k, J^{-1} in the last pass;
    # phi with its i derivatives (Q in, 4 + 4 out), the j and k derivatives (4 in, 4 out each); per direction
    # the viscous faces and differences (phi 4 + derivatives 8 + face metrics 7 + S_d 3 + J^{-1} 1 in, r 4 in
    # and out), the last one applying the RK3 stage (R_rho 1, Q 5 and Q^n 5 in, Q 5 out).
    per_cell = 8 * ((3 * 5 + 3 * 3 + (5 + 2 * 5 + 2 * 5) + 1) + (5 + 8) + 2 * (4 + 4)
                    + 3 * (4 + 8 + 7 + 3 + 1 + 4 + 4) - 4 + (1 + 5 + 5 + 5))
    achieved = per_cell * cells * 3 / (ms / 1e3) / 1e9
    print(json.dumps({
        "metric": "Mcell-stage/s of RK3 Navier-Stokes steps of the paper's operator (WCNS-E-5 + fourth-order "
                  "viscous) on the one-GPU share's geometry closed at the wall and far field",
        "value": round(cells * 3 / (ms / 1e3) / 1e6, 1), "unit": "Mcell-stage/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (uniform stream at M 0.8)",
        "config": {"workload": f"ns_wcns5_c4_share_{nb}x{nb}_of_{ni}x{nj}x{nk}", "cells": cells,
                   "blocks": len(tl.owners), "ghost_blocks": 2 * len(tl.owners), "setup_s": round(setup_s, 1),
                   "finite": finite},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "algorithmic_bytes_per_cell_stage":
                     per_cell, "kernel": "pipeline: k_wcns5_euler_rows, k_wcns5_euler_march<1|2>, k_c4_phi_grads_i, "
                     "k_c4_grads_march<1|2>, k_c4_visc_rows, k_c4_visc_march<1, false>, k_c4_visc_march<2, true>"},
        "cpu_baseline": None}), flush=True)
    return 0


def bench_mg_channel(a) -> int:
    """Multigrid V-cycles of the steady march (three levels, one RK3 step on
    each finer level, two on the coarsest) on the 192 x 96 x 96 channel with
    a bump at M 0.6 (the warm-start family's grid): K cycles after W warm-up
    ones, one cfd_mg_cycles call, hipEvents on the launch stream, no history
    kept.  The state drifts toward the steady flow while it is timed; the
    cycle's work does not depend on it.  --tune picks each level's tiles
    first (autotune_multigrid, on a scratch copy of the state)."""
    import torch
    from paper_1710_09995_amd import cases
    from paper_1710_09995_amd.binding import Multigrid, Solver
    case = cases.channel_case(192, 96, 96, mach=0.6, hb=0.05)
    s = Solver(case)
    mg = Multigrid(s, 3, 1, 2)
    tune_info = None
    if a.tune:
        from paper_1710_09995_amd.autotune import autotune_multigrid
        res = autotune_multigrid(mg, log=lambda m: print(m, file=sys.stderr, flush=True))
        tune_info = {"levels": res["tunings"], "ms_per_cycle_tuning": round(res["ms_per_cycle"], 4),
                     "candidates": len(res["table"])}
        print(f"# tuned: {res['tunings']} ({res['ms_per_cycle']:.4f} ms/cycle)", file=sys.stderr, flush=True)
    mg.cycles(a.warmup, hist=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    mg.cycles(a.steps, hist=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    cells = 192 * 96 * 96
    print(json.dumps({
        "metric": "fine-grid Mcell-cycle/s of three-level multigrid V-cycles (RK3 smoother) on the channel",
        "value": round(cells / (ms / 1e3) / 1e6, 1), "unit": "Mcell-cycle/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (channel with a bump, M 0.6)",
        "config": {"workload": "mg_channel_192x96x96_3levels_pre1_coarse2", "cells": cells,
                   "tuning": [lv.get_tuning() for lv in mg.levels], "autotune": tune_info,
                   "finite": bool(all(torch.isfinite(v).all() for v in s.interior_views()))},
        "roofline": None, "cpu_baseline": None}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="paper_share", choices=["bump_ns", "vortex", "batched", "paper_share"])
    ap.add_argument("--reps", type=int, default=5, help="timed runs of K steps; value = the best (paper protocol)")
    ap.add_argument("--no-fp32-check", action="store_true",
                    help="skip the FP32-flux rerun and its L2 error against the FP64 state")
    ap.add_argument("--flux", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--kernel", type=int, default=None)
    ap.add_argument("--tile-j", type=int, default=None)
    ap.add_argument("--tile-k", type=int, default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--order", type=int, default=None, choices=[0, 1], help="tile order (1 = XCD-aware)")
    ap.add_argument("--tune", action="store_true",
                    help="run the tile autotuner first (default: the library's default tiles)")
    ap.add_argument("--no-tune", action="store_true", help="accepted for compatibility; the default")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--split", type=int, default=0, metavar="MAX_CELLS",
                    help="cut the blocks into pieces of at most MAX_CELLS cells first (Section 3.2.1)")
    ap.add_argument("--split-align", default="64,8,1", metavar="I,J,K",
                    help="with --split: cut positions snap to multiples of these (1,1,1 = plain bisection)")
    ap.add_argument("--groups", type=int, default=8,
                    help="with --split: groups (devices) the pieces are regrouped into for the balance report")
    ap.add_argument("--op", default=None, choices=["diff6", "wcns5", "wcns5_euler", "ns_periodic", "wcns5_curv", "ns_curv", "implicit_curv",
                             "ns_blocks", "ns_share", "mg_channel"],
                    help="time one operator instead of the solver, on a 256x128x128 block, 5 variables, each "
                         "direction: diff6 = the sixth-order staggered flux difference (Section 2.2, Eq. 2); "
                         "wcns5 = the WCNS-E-5 weighted cell-edge interpolation; wcns5_euler = the periodic "
                         "inviscid WCNS-E-5 residual (all three directions); ns_periodic = that residual plus the "
                         "fourth-order central viscous terms; wcns5_curv = the inviscid residual on a wavy "
                         "curvilinear periodic grid (metrics computed once, their time reported); ns_curv = that "
                         "residual plus the curvilinear fourth-order viscous terms; implicit_curv = implicit "
                         "steps (backward Euler, Jacobi sweeps) on the curvilinear residual; ns_blocks = RK3 "
                         "Navier-Stokes steps on that grid cut into 2 x 2 x 2 blocks joined face to face, with the "
                         "unsplit block timed beside it; ns_share = RK3 Navier-Stokes steps on 2 x 2 of the one-GPU "
                         "share's 512x512x144 blocks closed at the wall and far field; mg_channel = three-level "
                         "multigrid V-cycles on the 192x96x96 channel (a cycle is a step)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (HBM counter calibration) and exit")
    a = ap.parse_args(argv)
    if a.calibrate_copy:
        import torch
        n = a.calibrate_copy * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 5}), flush=True)
        return 0
    if a.op in ("wcns5_euler", "ns_periodic", "wcns5_curv", "ns_curv") and a.gpus == 1:
        return bench_wcns5_euler(a)
    if a.op == "implicit_curv" and a.gpus == 1:
        return bench_implicit(a)
    if a.op == "ns_blocks" and a.gpus == 1:
        return bench_ns_blocks(a)
    if a.op == "ns_share" and a.gpus == 1:
        return bench_ns_share(a)
    if a.op == "mg_channel" and a.gpus == 1:
        return bench_mg_channel(a)
    if a.op is not None and a.gpus == 1:
        return bench_op(a)
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(sharding across GPUs is a design note, not code); use --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_1710_09995_amd.binding import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev_inputs = "cuda:0" if a.workload == "paper_share" else None
    case, label = make_case(a.workload, a.flux, device=dev_inputs)
    print(f"# workload {label}: {case.nblk} blocks, {case.ncells} cells, flux {a.flux}", file=sys.stderr,
          flush=True)
    split_info = None
    if a.split:
        from paper_1710_09995_amd import partition as part

        def balance(loads):
            _, tot = part.regroup(loads, a.groups)
            return round(max(tot) / (sum(tot) / a.groups), 4)

        blocks_loads = [ni * nj * nk for ni, nj, nk in case.dims]
        align = tuple(int(v) for v in a.split_align.split(","))
        case, pieces = part.split_case(case, a.split, align=align)
        split_info = {"max_cells": a.split, "align": list(align), "blocks": len(blocks_loads), "pieces": len(pieces),
                      "groups": a.groups, "max_over_mean_blocks": balance(blocks_loads),
                      "max_over_mean_pieces": balance([p.cells for p in pieces])}
        print(f"# split: {json.dumps(split_info)}", file=sys.stderr, flush=True)
    s = Solver(case, device="cuda:0")
    tun = {}
    if a.kernel is not None:
        tun["kernel"] = a.kernel
    if a.tile_j is not None:
        tun["tile_j"] = a.tile_j
    if a.tile_k is not None:
        tun["tile_k"] = a.tile_k
    if a.no_graph:
        tun["use_graph"] = 0
    if a.order is not None:
        tun["order"] = a.order
    tune_info = None
    if tun:
        s.set_tuning(**tun)
    elif a.tune:
        from paper_1710_09995_amd.autotune import autotune
        res = autotune(s, log=lambda m: print(m, file=sys.stderr, flush=True))
        tune_info = {"cached": res["cached"], "ms_per_step_tuning": round(res["ms_per_step"], 4),
                     "candidates": len(res["table"])}
        print(f"# tuned: {res['tuning']} ({res['ms_per_step']:.3f} ms/step)", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    s.step(a.warmup, hist=False)
    torch.cuda.synchronize()
    reps = [timed_steps(torch, s, a.steps, stream) for _ in range(max(1, a.reps))]
    for r, m in enumerate(reps):
        print(f"# run {r}: {a.steps} steps in {m:.2f} ms", file=sys.stderr, flush=True)
    ms = min(reps)
    ms_median = float(sorted(reps)[len(reps) // 2]) if len(reps) % 2 else 0.5 * sum(sorted(reps)[len(reps) // 2 - 1:
                                                                                            len(reps) // 2 + 1])
    cell_stages = case.ncells * 3 * a.steps
    value = cell_stages / (ms / 1e3) / 1e6
    h = s.step(1, hist=True).cpu().numpy()[0]
    finite = bool(all(math.isfinite(x) for x in h))

    roofline = None
    fp64 = None
    prof = None
    if not a.no_profile_pass:
        s.set_profiling(True)
        s.step(a.steps, hist=False)
        torch.cuda.synchronize()
        prof = s.profile_read()
        s.set_profiling(False)
        st = prof["stage"]
        bpc = stage_bytes_per_cell(bool(case.params.local_dt))
        per_launch = bpc * case.ncells
        achieved = per_launch / (st["mean_ms"] / 1e3) / 1e9
        kernel_label = f"stage_{label}_{a.flux}" + (f"_split{a.split}" if a.split else "")
        traffic = read_traffic(kernel_label)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": {0: "k_stage_tiled", 1: "k_stage_simple", 2: "k_stage_ring"}.get(
                        s.get_tuning()["kernel"], "k_stage") + " (residual + RK stage update)",
                    "mean_launch_ms": round(st["mean_ms"], 4), "launches": st["launches"],
                    "algorithmic_bytes_per_cell": round(bpc, 2), "cells_per_launch": case.ncells}
        flops = read_profile_value(kernel_label, "valu", "fp64_flops_per_launch")
        if flops is not None:
            tf = flops / (st["mean_ms"] / 1e3) / 1e12
            fp64 = {"achieved": round(tf, 2), "peak": FP64_VECTOR_PEAK, "unit": "TFLOP/s",
                    "frac": round(tf / FP64_VECTOR_PEAK, 4), "flops_per_launch": flops,
                    "flops_per_cell": round(flops / case.ncells, 1),
                    "note": "executed FP64 flops from SQ_INSTS_VALU_*_F64 counters (profiles/*_valu.txt), "
                            "incl. reciprocal/sqrt refinement"}
        print(f"# profile: {json.dumps(prof)}", file=sys.stderr, flush=True)
    tune = s.get_tuning()
    fp32_check = None
    if a.flux == "fp64" and not a.no_fp32_check and split_info is None:
        fp32_check = fp32_flux_check(torch, s, case, a, stream,
                                     lambda: make_case(a.workload, "fp32", device=dev_inputs)[0])
    s.close()
    del s

    cpu = None
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.workload, a.flux, a.cpu_budget)

    out = {
        "metric": "Mcell-stage updates/s + % HBM peak; wall-clock to 1e-8 residual drop",
        "value": round(value, 2),
        "unit": "Mcell-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.flux == "fp64" else "f32-flux/f64-state",
        "data": "synthetic (seeded grid, state and noise)",
        "config": {"workload": label, "blocks": case.nblk, "cells": case.ncells,
                   "viscous": bool(case.params.viscous), "flux": a.flux, "stages_per_step": 3,
                   "tuning": tune, "autotune": tune_info, "finite": finite, "split": split_info,
                   "inputs": "generated on the device" if dev_inputs else "generated on the host",
                   "protocol": {"runs": len(reps), "value_is": "best run",
                                "ms_per_step_runs": [round(m / a.steps, 4) for m in reps],
                                "median_ms_per_step": round(ms_median / a.steps, 4),
                                "value_median": round(cell_stages / (ms_median / 1e3) / 1e6, 2)},
                   "fp32_flux_check": fp32_check},
        "roofline": roofline,
        "fp64_valu": fp64,
        "cpu_baseline": cpu,
    }
    if prof is not None:
        out["kernel_ms"] = {k: {"mean": round(v["mean_ms"], 4), "launches": v["launches"]} for k, v in prof.items()}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
