"""FP64 CPU oracle for overrelaxation gauge fixing (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the HIP product path and imports
nothing from it.

* ``gf_oracle.c`` -- Alg. 1 (overrelaxation with even/odd sites), eqs. (1)-(6),
  reunitarisation; plain C99 loops in double precision.
* ``gf_oracle_sun.c`` / ``sun.py`` -- the same for SU(N), N >= 2 (all N(N-1)/2
  SU(2) subgroups).
* ``diff.py`` -- the functional F_U[g] as a function of g(x) = exp(S(x)) and its
  gradient by eigendecomposition (numpy), plus the steepest-descent step of
  eq. (7).
"""
from .core import (  # noqa: F401
    build, load, quality, divergence_field, staple, su2_solve,
    subgroup_update, site_update, half_sweep, half_sweep_order, sweep,
    reunit, fix, parity_of_sites, set_threads,
)
from . import sun  # noqa: F401
