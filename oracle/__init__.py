"""Plain CPU float64 oracle for the ADI isogeometric Maxwell time step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
GPU library never calls it, links it or shares code with it; the only
thing both sides share is the seeded input generator module
``workloads`` (which contains none of the method's arithmetic).

The oracle follows the paper (Paszynski, Los, Munoz-Matute, "Alternating
directions implicit higher-order finite element method for simulations
of time-dependent electromagnetic wave propagation in non-regular
biological tissues", arXiv 2103.06998) step by step, in NumPy float64,
without any blocking or fusion:

* ``bspline``  -- open uniform knot vectors, Cox-de Boor B-splines and
                  their derivatives, Greville abscissae.
* ``gram``     -- the 1D mass, stiffness and advection matrices M, S, A, B
                  (section "Variational formulation", the matrix list after
                  eqs. discrete1-discrete4).
* ``banded``   -- pivot-free banded LU and the direction-wise line solves
                  (section "Incorporating non-regular material data ...").
* ``maxwell``  -- the two-substep ADI scheme, eqs. scheme1a-scheme1d /
                  weak1-weak4 / discrete1-discrete4, with test-function-wise
                  material.
* ``mms``      -- the manufactured solution u_A and the L2 / H(curl) norms
                  (section "Numerical code verification ...").
* ``closure``  -- float64 reference of the small 3D convolutional closure
                  network (forward, backward, Adam).

Every function cites the passage it follows.  Readings of passages that are
silent, ambiguous or misprinted are listed in the module docstrings.
"""
