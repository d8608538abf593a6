"""GPU: what the trained warm-start network gains over the uniform-stream start.

Small version of the pipeline (32 coarse training cases of 24 x 12 x 12,
two held-out cases of 48 x 24 x 24): the network is trained by the library's
own forward/backward/Adam kernels on solutions the solver produced, and the
warm start must begin below the cold start's residual and reach the deepest
residual decade both starts reach in fewer steps.  The network's output has
no closed form (parity unpinned); the residual history decides.
"""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_warm_start_beats_cold_start():
    from paper_1710_09995_amd import cases, warmstart
    data = warmstart.generate(32, seed=0, dims=(24, 12, 12), drop=1e-12, max_steps=3000)
    say("data", data.x.shape[0], "points, residual", data.info["r0"], "->", data.final_residual)
    assert data.final_residual < 1e-2 * data.info["r0"]
    net = warmstart.train(data, iters=800, batch=4096)
    tests = cases.channel_conditions(2, 12345)
    res = warmstart.compare(net, tests, dims=(48, 24, 24), max_steps=4000, log=say)
    for c in res:
        assert c.r_warm0 < c.r_cold0
        d = warmstart.deepest_common(c)
        assert d is not None
        say(f"  M={c.mach:.3f}: deepest common drop {d:.0e}: cold {c.cold[d][0]} steps, warm {c.warm[d][0]} steps")
        assert c.warm[d][0] < c.cold[d][0]
        assert np.isfinite(c.warm_final) and c.warm_final <= c.cold_final * 1.5
