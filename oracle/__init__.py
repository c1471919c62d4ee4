"""Plain FP64 CPU oracle for the adjoint-descent method of Ashtari & Schneider
(arXiv 2306.00165) applied to plane Couette flow.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_2306_00165_amd/``), and the HIP path never imports it.

What it computes, each piece written from the paper's definitions with dense
per-Fourier-mode matrices and library FFTs, no blocking or fusion:

* ``cheb``   -- Chebyshev collocation/coefficient operators in y
                (Sec. 4, Fourier-Chebyshev-Fourier expansion).
* ``grid``   -- the discretisation: retained Fourier modes, box, Re, Delta t.
* ``flow``   -- the dealiased convective term of the perturbative NSE
                (Sec. 3.1, momentum equation with u_b = y e_x from Sec. 5)
                and its linearisation, plus their exact W-adjoints.
* ``stokes`` -- the implicit Stokes step solved as the dense Chebyshev-tau
                system (Sec. 4, steps (1)-(3): one first-order IMEX step that
                keeps the velocity divergence-free and no-slip).
* ``method`` -- residual r(u), cost J^2 = <r, r> (Sec. 2, Sec. 3.2),
                directional derivative and its adjoint (Sec. 3.3, App. A),
                the L2-orthogonal projection onto divergence-free no-slip
                fields (Sec. 3.4), the forward-Euler descent (Sec. 4,
                step (5)), diagnostics and the minimal real state vector
                (Sec. 6.2).
* ``dmd``    -- dynamic mode decomposition and extrapolation (Sec. 6).
* ``mlp``, ``pod`` -- the learned extrapolator that sits beside DMD: a
                bfloat16-quantised multilayer perceptron with back-propagation
                and Adam, and the POD of snapshot sets.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
library routines, brute force on tiny grids and invariants of the method.
"""

from .grid import Grid  # noqa: F401
from . import cheb, flow, stokes, method, state, dmd, mlp, pod  # noqa: F401
