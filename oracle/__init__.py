"""FP64 CPU oracle for the relativistic quasiparticle lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may use it.  It shares no code with the HIP path.

It is a plain, slow, vectorised-over-sites numpy implementation of what the
paper (P. Romatschke, "Relativistic (Lattice) Boltzmann Equation with
Non-Ideal Equation of State", arXiv:1108.5561) computes:

* ``quadrature``  - the momentum lattice of Sec. IV.C (phi nodes, Gauss-Legendre
  polar nodes, radial nodes from the polynomials R_k orthogonal on
  exp(-z0 cosh xi) sinh^2 xi).
* ``eos``         - the quasiparticle equation of state of Sec. III and III.A
  (M(T) from the entropy, B(T), eqs. (epsp), (cdef2)) and the BGK relaxation
  time from the Chapman-Enskog shear viscosity of Sec. IV.A.
* ``lattice``     - node table, weights and the weak-form momentum-derivative
  operators S1, S2 of Sec. IV.D (projection onto L_m(cos theta) R_l(cosh xi)).
* ``force3d``     - the weak-form 3-D operator of the mass-gradient force on
  the test space of eq. (fansatz) (harmonics of v/|v| times powers of
  sinh xi times polynomials in cosh xi).
* ``step``        - one Heun (predictor / corrector) step of the Milne
  lattice-Boltzmann scheme of Sec. IV.D, extended to a periodic transverse
  (x, y) lattice; Landau matching of eq. (sanity).
* ``bjorken``     - the paper's own 0+1-D algorithm of Sec. IV.D, written
  separately (homogeneous medium, U = (1, 0, 0, 0)).
* ``hydro``       - fluid-dynamics reference ODEs (ideal and first-order
  viscous Bjorken flow; eq. (hydroeq)).

Every function cites the passage it follows.  Readings of passages that are
silent, garbled or ambiguous are listed in the docstrings where they are used.
"""
