"""Plain FP64 CPU oracle for the FB-LTS hot path (test infrastructure only).

This package is the slow, obviously-correct reference the HIP library is
checked against.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the product path never does.  It
shares no code with the HIP library: both only read the same mesh arrays and
the same seeded inputs.

Every function follows a passage of the paper (Lilly, Capodaglio, Engwirda,
Higdon, Petersen: "Local time-stepping for the shallow water equations using
CFL optimized forward-backward Runge-Kutta schemes", arXiv 2405.10505),
cited by section / equation label:

* ``trisk``   - TRiSK thickness tendency (eq. ``trisk_thickness``), momentum
  tendency in vorticity-flux form (eq. ``trisk_vorticity``, eq.
  ``nonlinear_swe``; drag and wind stress of eq. ``hurricane_model``),
  diagnostics of Section 2.4.
* ``schemes`` - FB-RK(3,2) (eq. ``fbrk32``), RK4, RK(3,2), and the FB-LTS
  step of Section 2.2 (coarse advancement, interface prediction eq. ``preds``,
  fine advancement eq. ``fine_fbrk32``, interface correction eq.
  ``if_correction``).
* ``regions`` - the LTS regions of Section 2.2 (fine, interface one/two,
  interior coarse; the interface-adjacent fine layers F^l).

Parity pins: see the module headers.  The quadratic drag and wind-stress terms
(eq. ``hurricane_model``) follow a reading of the paper.  Their vector laws are
pinned by closed forms for uniform flow (tendencies on the regular hexagon, and
an inertial oscillation with quadratic drag), the edge value of a varying C_D
by a linear field on the hexagon.  The coefficients C_D (per cell) and C_W (per
edge, from the wind through Garratt's law) are inputs, like the wind itself.
"""
from . import trisk, schemes, regions  # noqa: F401
