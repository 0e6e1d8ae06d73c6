"""CPU FP64 oracle for the Wilson-Dirac operator and its CG solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_1810_04201_amd``) and imports nothing
from it; both sides take their seeded inputs from ``synth``.

Everything is plain NumPy in complex128, written from the paper
("Towards Lattice Quantum Chromodynamics on FPGA devices", Korcyl & Korcyl):

* ``gamma``   -- the Dirac matrices of Appendix A (Conventions).
* ``wilson``  -- the operator of Eq. (1) of Sec. 2.1 and its adjoint, as a
                 whole-lattice stencil (np.roll) and at chosen sites.
* ``dense``   -- the same operator assembled entry by entry as a dense
                 12V x 12V matrix (tiny lattices only).
* ``cg``      -- conjugate gradient of Sec. 2.2 on the normal equations.
* ``free``    -- the free-field (U = 1) operator in momentum space.
* ``gauge``   -- gauge transformations (covariance pin).

Readings adopted where the paper is silent or garbled are stated in each
function's docstring (sign of the hopping term, the backward link index,
normal-equation form, squared norms in the CG listing, stopping rule,
antiperiodic time direction).
"""
from . import gamma, wilson, dense, cg, free, gauge  # noqa: F401
