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
mlp        FP64 multilayer perceptron forward/backward (warm start)
partition  block split plan, split tables, LPT regroup (Section 3.2.1)
highorder  sixth-order staggered flux difference (Section 2.2, Eq. 2)

Parity status: every function is pinned by the CPU tests (closed forms,
invariants, textbook special cases, brute force) except the trained
warm-start network's output, which has no closed form ("parity unpinned";
it is assessed by residual history only).
"""
from . import geometry, ghosts, flux, solver  # noqa: F401
