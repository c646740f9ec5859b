"""CPU oracle for the coupled spin-torque-oscillator reservoir.

TEST INFRASTRUCTURE.  This package is the plain, slow, FP64 reference that
the HIP library is checked against.  It may be imported, called or executed
only by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline
leg of ``bench.py``.  The product library never imports, links or calls it,
and it shares no code, header, table or constant with the HIP path; only
the seeded input generators in ``workloads/`` feed both.

Contents (paper citations by section and equation):

* ``constants``: Table 1 and its dimensionless form;
* ``sto``: the right-hand side of Eq. (gov) with Eq. (coup) and Eq. (in),
  classic RK4 (Sec. 3.2), records per input sample, Lyapunov estimate;
* ``readout``: ridge-regression readout (the paper trains only the readout,
  Sec. 1; the algorithm is this oracle's reading);
* ``exactdot.c``: correctly rounded dot products (plain C, gcc), which fix
  the rounding of the coupling and input sums.

Every function is pinned by the ``-m "not gpu"`` tests against closed forms,
invariants and brute force.  The coupled, driven trajectory values
themselves have no printed values in the paper; they are pinned only
through those checks of the pieces that produce them.
"""

from . import constants, readout, sto  # noqa: F401
from ._native import build as build_native  # noqa: F401
from ._native import exact_dot, exact_matvec, exact_sum  # noqa: F401
