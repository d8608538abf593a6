"""The allocation-free entry point cfd_wcns5_euler_residual_periodic_noalloc
(its scratch is the library's static device array) against the entry point
that takes a workspace, cfd_wcns5_euler_residual_periodic, through the C ABI:
two calls in a row, the second on a smaller block, each bitwise equal to the
workspace entry point (the same kernels on the same launch shapes) and within
the FP64 gate of the oracle's residual; a block too large for the static
array is refused before any launch."""
import numpy as np
import pytest

from gpu_util import say
from oracle import highorder as ho

pytestmark = pytest.mark.gpu


def _state(n, seed):
    """A periodic flow with smooth waves and seeded cell noise (every
    component varies along every axis; density and pressure stay positive)."""
    ni, nj, nk = n
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)
    z, y, x = np.meshgrid(np.arange(nk) / nk, np.arange(nj) / nj, np.arange(ni) / ni, indexing="ij")
    s = 2 * np.pi
    rho = 1 + 0.2 * np.sin(s * x + ph[0]) * np.cos(s * y + ph[1]) + 0.1 * np.sin(s * z + ph[2])
    u = 0.5 + 0.1 * np.sin(s * y + ph[3])
    v = -0.2 + 0.1 * np.sin(s * z + ph[4])
    w = 0.1 * np.sin(s * x + ph[5])
    p = 1 + 0.1 * np.cos(s * (x + y + z))
    rho = rho * (1 + 0.01 * rng.uniform(-1, 1, rho.shape))
    p = p * (1 + 0.01 * rng.uniform(-1, 1, p.shape))
    return np.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)])


def test_noalloc_residual_matches_workspace_entry_point_twice():
    import torch
    from paper_1710_09995_amd.binding import (wcns5_euler_residual_periodic,
                                              wcns5_euler_residual_periodic_noalloc)
    for call, n in enumerate([(72, 40, 28), (37, 9, 13)]):     # second call: a smaller block
        say("noalloc residual call", call, "n", n)
        q = _state(n, seed=11 + call)
        h = (2.0 / n[0], 1.5 / n[1], 1.0 / n[2])
        qd = torch.from_numpy(q).cuda()
        out = torch.full_like(qd, float("nan"))
        wcns5_euler_residual_periodic_noalloc(qd, h, out)
        ref = wcns5_euler_residual_periodic(qd, h)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want_ws = ref.cpu().numpy()
        assert np.array_equal(got, want_ws), "no-alloc residual differs from the workspace entry point"
        want = ho.wcns5_euler_residual_periodic(q, h, 1.4, 0.1)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        say("  max |R - R_oracle| / max |R_oracle| =", f"{err:.2e}")
        assert err <= 1e-12


def test_noalloc_residual_refuses_a_block_beyond_its_scratch():
    import torch
    from paper_1710_09995_amd.binding import CfdError, wcns5_euler_residual_periodic_noalloc
    n = (128, 128, 96)                  # needs about 135 MB of scratch, over the 64 MiB array
    q = torch.ones((5, n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(q)
    with pytest.raises(CfdError, match="CFD_WCNS5_NOALLOC_MAX_BYTES"):
        wcns5_euler_residual_periodic_noalloc(q, (0.1, 0.1, 0.1), out)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0          # nothing was launched
