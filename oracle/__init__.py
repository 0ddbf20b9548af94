"""Plain FP64 CPU oracle for the continuous-field DQMC sweep of the projected
SO(5) model (arXiv 2605.03700).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the bench's CPU-baseline leg may import it. The GPU library never calls it and
shares no code, tables or constants with it.

Every function cites the passage of the paper it follows (section, equation).
The oracle computes per-configuration quantities by their plain definitions
(dense products, inverses and determinants) and runs the Markov chain in the
order the paper's Methods section states. Readings of silent or garbled
passages are listed in the design notes of the repository.

Parity status per module:
  model.py        pinned (Fock-space construction, Hermiticity, counts; the
                  torus density operator against the overlap integrals of the
                  printed LLL wave functions over one periodic cell)
  fock.py         pinned (Fierz identity exact on one orbital; HS quadrature)
  dqmc.py         pinned (closed forms, Fock-trace identity, mpmath brute
                  force, finite-difference gradient, Gaussian MALA limit;
                  the interacting chain at N = 2, L = 1: every ln A against
                  its closed form, the stationary law against quadrature,
                  the step-size controller settling at the set point)
  observables.py  pinned (Fock-space expectation values at small size)
  slmc.py         pinned (Parseval, closed-form periodogram, translation
                  invariance, finite differences, torch bfloat16 and Adam,
                  leapfrog reversibility, stationary law of the global move)
"""
