"""Test-only FP64 CPU oracle for the orthogonal discrete spherical Bessel transform.

This package is test infrastructure.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product library
(``paper_1509_07115_amd``) never imports, links or executes anything here, and
this package imports nothing from the product.

Modules
-------
dsbt     dense FP64 transform built straight from the definitions (Sec. 2.2-2.5)
exact    exact-rational (``fractions``) DLOP / DDLOP / T for tiny grids (Sec. 2.3-2.5, App. A)
tdse     dense split-operator step, propagation and adjoint gradient (Sec. 4.1)
sbf      spherical-Bessel references: closed forms, quadrature, corrected momenta (Sec. 3)
monomial the paper's own monomial-moment fast multiplication (Sec. 2.6), FP64, for its error envelope
angular  the angular transform Y = P Phi of the DSBT-DVR solver (Sec. 4.1)
tdse3d   dense 3D split step in the coordinate gauge (Sec. 4.1) for the oscillator test of Sec. 4.2
"""
from . import dsbt, exact, tdse, sbf, monomial, angular, tdse3d  # noqa: F401
