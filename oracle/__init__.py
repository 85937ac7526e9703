"""FP64 CPU oracle for the MGRIT / eddy-current hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; both read
the same seeded inputs from the `workload` package and nothing else.

Every routine is a plain, slow, obviously checkable restatement of the paper
(arXiv:1912.03106) or of textbook finite elements, in float64, using SciPy's
sparse LU as the linear-solve primitive:

  pwm.py       PWM excitation, Sec. 3.2 and Sec. 3.3 (reference signals and
               carrier equations)
  fe.py        P1 finite elements for the eddy-current problem, Sec. 3.1
               (semi-discrete system, eq. 7) and the saturating reluctivity
  stepping.py  implicit Euler propagator Phi (eq. 8, eq. 2) with direct solves
               and Newton, sequential forward solve (Sec. 2)
  transfer.py  spatial interpolation / restriction between nested meshes
               (Sec. 2.2, Sec. 3.4)
  mgrit.py     FAS-MGRIT (Algorithm 1), V-cycle recursion (Sec. 2.1), Parareal
               (the two-level F-relaxation special case)

Readings of points the paper leaves open are listed in the design notes; each
function states the one it uses.
"""
