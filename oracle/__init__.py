"""CPU FP64 oracle for the matrix-free Lippmann-Schwinger (LS) displacement operator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never routes through
it, and this package shares no code with that path: it is a plain, slow,
directly checkable restatement of the method of Shekhar, Jakobsen, Iversen,
Berre and Radu, "Integral equation method for microseismic wavefield modelling
in anisotropic elastic media" (arXiv 2301.12836):

* ``oracle.green``    - the background elastodynamic Green's tensor (Eq 7,
  Appendix A: A.4, A.5 and the derivative formulas A.6-A.11) and the r = 0
  self-term.
* ``oracle.operator`` - the discrete operator of Eq 19-21: the finite-difference
  strain of Eq 17-18, the Voigt contrast product of Eq 11-12, the Green's tensor
  convolution, the moment-tensor incident field of Eq 13-16; dense assembly,
  brute-force O(n^2) apply and a zero-padded FFT apply.
* ``oracle.solve``    - the dense direct solve and a textbook BiCGSTAB with the
  relative residual of Eq 22.
* ``oracle.adjoint``  - the transposed operator, receiver sampling and the dense
  adjoint-state gradient of a receiver misfit.
* ``oracle.synthesis`` - the Ricker wavelet of Tables 1 and 3, its spectrum,
  and time-domain traces from one-sided frequency-domain solutions.

Everything is float64 / complex128.  Arrays use the layout
``u[3][N3][N2][N1]`` (component, z, y, x), contrast ``dC[21][N3][N2][N1]``
(Voigt upper triangle, row order 11,12,...,16,22,...,66), ``drho[N3][N2][N1]``.

Parity status: the Green's tensor, self-term, strain operator, contrast
product, incident field and operator are pinned by tests under
``tests/test_oracle_*.py`` (closed forms, textbook limits, reciprocity, the
Born limit, uniform-contrast physics and three independent constructions of the
operator).  The paper prints no numerical values for any worked example (its
figures are placeholders), so no pin compares against a printed number.
"""

from . import adjoint, green, operator, solve, synthesis  # noqa: F401
