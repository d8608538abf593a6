"""Writes c3_seed0_dt.txt: the oracle's global CFL time step of the 64-block
batched Euler workload (block extents drawn from [16, 160], seed 0, FP64
flux) at its initial state, and every block's least per-cell step.

The step of a cell (the reading of the step size that Eqs. 4-6 leave open:
CFL V over the sum of the spectral radii along the three directions) reads
only the cell's own state, its six face vectors and its volume, all of which
come from the block's own nodes.  Each block is therefore evaluated alone,
which keeps the oracle's memory to one block at a time; it gets far field on
its six faces, so that its ghost nodes are extrapolated (no interior cell's
step reads them).  Calls only the oracle and the seeded input generator.

Usage (repo root): python tests/golden/make_c3_seed0_dt.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import solver as osol  # noqa: E402
from paper_1710_09995_amd import cases  # noqa: E402


def main():
    c = cases.batched_euler_case(64, seed=0, flux_fp32=0)
    per_block = []
    for b in range(c.nblk):
        bcs = [cases.full_bc(0, c.dims[b], face, cases.FARFIELD) for face in range(6)]
        one = cases.Case("block", c.params, [c.dims[b]], [c.nodes[b]], [], bcs, [c.q0[b]])
        st = osol.setup(one)
        dt = osol.local_dt_block(st.Qs[0], st.Ss[0], st.Vs[0], c.dims[b], c.params, st.g)
        per_block.append(float(dt.min()))
        print(f"block {b}: {c.dims[b]} least dt {per_block[-1]!r}", flush=True)
    with open(os.path.join(HERE, "c3_seed0_dt.txt"), "w") as f:
        f.write("# Oracle CFL time step of the 64-block batched Euler workload, seed 0, at its initial state\n")
        f.write("# (written by tests/golden/make_c3_seed0_dt.py; FP64, CFL 0.5, Mach 0.5)\n")
        f.write(f"dt_global {min(per_block)!r}\n")
        for b, v in enumerate(per_block):
            f.write(f"block {b} {v!r}\n")


if __name__ == "__main__":
    main()
