"""Shared helpers of the GPU parity tests (oracle vs the HIP path on the same
seeded inputs)."""
import sys

import numpy as np

from oracle import solver as osol
from paper_1710_09995_amd import cases


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a_list, b_list):
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(b ** 2)) for b in b_list)
    return (num / den) ** 0.5


def max_rel(a_list, b_list):
    num = max(float(np.max(np.abs(a - b))) for a, b in zip(a_list, b_list))
    den = max(float(np.max(np.abs(b))) for b in b_list)
    return num / den


def small_cases():
    """Parity workloads sized for the oracle (seconds), several tiles with ragged tails."""
    out = {}
    out["vortex16"] = cases.vortex_case(16, seed=1)
    out["vortex_curv"] = cases.vortex_case(20, nz=12, seed=2, curvilinear=True)
    out["bump_ns"] = cases.bump_ns_case(70, 20, 12, seed=3, noise=1e-3, reynolds=5e3)
    out["batched"] = cases.batched_euler_case(nblk=5, seed=4, lo=6, hi=23, flux_fp32=0)
    ch = cases.channel_case(40, 12, 6, mach=0.7, hb=0.08)
    out["channel_local"] = ch
    return out


def oracle_steps(case, n):
    st = osol.setup(case)
    rows = [osol.step(st, record=True) for _ in range(n)]
    return osol.interior_state(st), rows


def oracle_residual(case):
    st = osol.setup(case)
    return osol.residual(st)
