"""Sixth-order staggered flux difference (oracle; plain FP64 NumPy).

Test infrastructure, like the rest of this package.

Section 2.2, Eq. (2): the cell-centred derivative of a face-centred flux F
along one index direction with grid size h,

    dF/dxi |_i = [ 75/64  (F_{i+1/2} - F_{i-1/2})
                 - 25/384 (F_{i+3/2} - F_{i-3/2})
                 +  3/640 (F_{i+5/2} - F_{i-5/2}) ] / h.

The face field holds n + 5 faces along the direction (faces i - 1/2 for
i = -2 .. n + 2), so every one of the n cells has its six faces.  How the
faces beyond a block are obtained (ghost cells, boundary closures) is in
references the paper does not reproduce; the operator takes them as given.

Pins: the printed weights' moment sums (exact rationals), exactness on
polynomials up to degree 6, the closed-form degree-7 error 225/64 h^6, and
sixth-order convergence on a sine.
"""
from __future__ import annotations

import numpy as np

C1, C2, C3 = 75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0


def staggered_diff6(f: np.ndarray, d: int, h: float) -> np.ndarray:
    """f: [nvar, Nk, Nj, Ni] face values with n_d + 5 entries along axis d
    (d = 0, 1, 2 for i, j, k); returns [nvar, nk, nj, ni] cell derivatives."""
    ax = 3 - d                       # array axis of direction d
    n = f.shape[ax] - 5

    def face(s):                     # faces i - 5/2 + s for the n cells
        sl = [slice(None)] * 4
        sl[ax] = slice(s, s + n)
        return f[tuple(sl)]
    c1, c2, c3 = C1 / h, C2 / h, C3 / h
    return c1 * (face(3) - face(2)) + c2 * (face(4) - face(1)) + c3 * (face(5) - face(0))
