"""GPU: what the trained warm-start network gains over the uniform-stream start.

Small version of the pipeline with the grid ratio of the full one (32 coarse
training cases of 24 x 12 x 12 marched to a 1e-8 drop, three held-out cases
of 48 x 24 x 24): the network is trained by the library's own
forward/backward/Adam kernels on converged solutions the solver produced.
Both starts march to one absolute target, 1e-8 of the cold start's initial
L2(R_rho), with the same steady march: plain local-step RK3 in one test, the
multigrid cycles the pipeline uses in the other.  The warm start (network
inference included) must reach the target in fewer steps or cycles on every
case and in fewer wall seconds over the median case.  The network's output
has no closed form (parity unpinned); the residual history decides.
"""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("levels", [1, 3])
def test_warm_start_reaches_the_target_sooner_than_the_cold_start(levels):
    from paper_1710_09995_amd import cases, warmstart
    data = warmstart.generate(32, seed=0, dims=(24, 12, 12), drop=1e-8, max_steps=40000 if levels == 1 else 5000,
                              levels=levels)
    say("data", data.x.shape[0], "points,", data.steps, "steps, residual", data.info["r0"], "->",
        data.final_residual)
    assert data.final_residual < 1e-8 * data.info["r0"]
    net = warmstart.train(data, iters=20000, batch=8192)
    tests = cases.channel_conditions(3, 12345)
    res = warmstart.compare(net, tests, dims=(48, 24, 24), max_steps=100000 if levels == 1 else 10000, log=say,
                            chunk=500 if levels == 1 else 100, levels=levels)
    T = warmstart.TARGET
    for c in res:
        assert T in c.cold and T in c.warm, (c.mach, c.hb)
        say(f"  M={c.mach:.3f} h={c.hb:.3f}: to {T:.0e}: cold {c.cold[T][0]} steps {c.cold[T][1]:.2f} s, "
            f"warm {c.warm[T][0]} steps {c.warm[T][1]:.2f} s (inference {c.inference_s * 1e3:.1f} ms)")
        assert c.r_warm0 < c.r_cold0
        assert c.warm[T][0] < c.cold[T][0]
    secs = warmstart.target_seconds(res)
    assert np.median([w for _, w in secs]) < np.median([c for c, _ in secs])


def test_warm_start_at_full_size():
    """The full sizes of the pipeline on one held-out case: 128 coarse training
    cases of 48 x 24 x 24 marched by multigrid cycles to a 1e-8 drop, the
    network trained on them, the first held-out condition of seed 12345 on
    192 x 96 x 96.  The warm start (inference included) reaches the 1e-8
    target in fewer cycles and fewer wall seconds than the cold start."""
    from paper_1710_09995_amd import cases, warmstart
    data = warmstart.generate(128, seed=0, dims=(48, 24, 24), drop=1e-8, max_steps=20000)
    say("data", data.x.shape[0], "points,", data.steps, "cycles", f"{data.seconds:.1f} s")
    assert data.final_residual < 1e-8 * data.info["r0"]
    net = warmstart.train(data, iters=20000, batch=8192)
    c, = warmstart.compare(net, cases.channel_conditions(1, 12345), dims=(192, 96, 96), max_steps=20000, log=say)
    T = warmstart.TARGET
    assert T in c.cold and T in c.warm
    say(f"  M={c.mach:.3f} h={c.hb:.3f}: cold {c.cold[T][0]} cycles {c.cold[T][1]:.2f} s, "
        f"warm {c.warm[T][0]} cycles {c.warm[T][1]:.2f} s")
    assert c.warm[T][0] < c.cold[T][0] and c.warm[T][1] < c.cold[T][1]
