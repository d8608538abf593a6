"""Plain FP64 CPU oracle for the structured-grid residual / RK3 path.

This package is test infrastructure.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library and its Python
binding never do.  It shares no code with the GPU path: it receives the seeded
inputs (nodes, connection and boundary tables, parameters, initial state) and
recomputes everything else itself.

Modules
-------
geometry   ghost nodes, face vectors and cell volumes (metrics)
ghosts     ghost-cell fill of the conserved state (connections and BCs)
flux       primitives, MUSCL reconstruction, Roe flux, viscous flux
solver     residual, time step, third-order Runge-Kutta, norms
implicit   backward-Euler steps with point-Jacobi sweeps on that residual
multigrid  full-approximation-storage V-cycles with the RK3 smoother
mlp        FP64 multilayer perceptron forward/backward (warm start)
partition  block split plan, split tables, LPT regroup (Section 3.2.1)
highorder  Section 2.2's operator: Eq. 2's sixth-order staggered flux
           difference, the WCNS-E-5 interpolation, residuals, viscous
           terms, metrics, RK3 and implicit steps on periodic and joined
           blocks
closures   walls and the far field for that operator (ghost blocks)

Parity status: every function is pinned by the CPU tests (closed forms,
invariants, textbook special cases, brute force), with these parts "parity
unpinned": the trained warm-start network's output (no closed form; the
residual history decides), the WCNS-E-5 nonlinear weights (from the
published scheme the paper cites; their linear limit, order, symmetry and
absence of overshoot are pinned), the multigrid cycle's correction scale
and restriction weights (they set how fast it converges, not where), and
how well the implicit steps' approximate Jacobian solves the exact linear
system (the operator itself is pinned).
"""
from . import geometry, ghosts, flux, solver  # noqa: F401
