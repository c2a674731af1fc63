"""Plain CPU oracle for the Leja phi-action path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The HIP library never calls it, and this package imports nothing
from the library: the two share no code.  Both take their inputs from the
seeded generators in ``paper_2310_08344_amd.workloads``, which hold none of the
method's arithmetic.

Everything is FP64 numpy, except the scalar phi functions and the Newton
divided differences, which are evaluated in mpmath at 50 significant digits
and rounded to FP64 once.

Modules
  leja        Leja points on [-2, 2], scalar phi_l, divided differences
  operators   periodic diffusion-advection and Burgers stencils
  phi_action  power iteration, the Newton-Leja loop, EXPRB42
  exact       references independent of Leja: dense augmented expm, FFT

Every function names the passage of the paper it follows (section, equation,
listing or table).  Where the paper is silent or garbled, the reading taken is
written out where it is used.
"""
