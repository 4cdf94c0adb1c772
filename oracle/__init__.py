"""Plain, slow, FP64 CPU oracle of the Hermite-leapfrog time step.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code,
table or constant with the HIP path (``paper_1808_10481_amd``) and imports
nothing from it; the product path never calls it.

The oracle follows Vargas, Hagstrom, Chan and Warburton, "Leapfrog
time-stepping for Hermite methods" (arXiv 1808.10481):

* ``hermite_lf``  - the scheme: Hermite-Birkhoff interpolation (Sec. 2,
  eq. (interp)), the leapfrog odd-term difference (Sec. 2, eqs. (option1),
  (option2), (update1)) with Cauchy-Kowalevsky exchange of time for space
  derivatives (Sec. 2, eqs. (LFloop), (final1); Sec. 3.1.2, eqs. (pdup),
  (vdup)), and the tensor-product extension (Sec. 5).
  Reflecting walls through mirrored ghost nodes (Sec. 5, "Imposing
  reflective boundary conditions"); the discrete adjoint of the periodic step
  (the transpose of the forward operators).
* ``diagnostics`` - error norms and the one-dimensional conserved quantity
  (Sec. 3.1.1, eqs. (Qdef), (Rdef), (fullcons1d)).

Every function is pinned by ``tests/test_oracle_*.py`` against facts the paper
and the mathematics fix; see the header of each module.
"""

from .hermite_lf import (  # noqa: F401
    Problem,
    hermite_matrix_exact,
    hermite_matrix,
    p_half,
    u_half,
    step,
    startup,
    p_update_cells,
    u_update_cells,
    ghost_pad,
    adjoint_step,
    kappa_gradient,
    adjoint_step_var,
    kappa_field_gradient,
    adjoint_step_var_bruteforce,
    kappa_field_gradient_fd,
    kmax_var,
    p_half_var,
    u_half_var,
    step_var,
    step_with_source,
    p_half_adjoint,
    u_half_adjoint,
    p_operator_blocks,
    u_operator_blocks,
)
from . import diagnostics  # noqa: F401
