"""Spherical-Bessel references for the DSBT oracle tests.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``gaussian_sbt``: closed form of the transform of eq. BesselProj for
  psi(r) = r^(l+1) exp(-a r^2) (the Gaussian atomic orbitals of Sec. 3):
  c_l(k) = k^(l+1) exp(-k^2/(4a)) / (2a)^(l+3/2).  It follows from the
  Hankel integral  int_0^inf r^(nu+1) J_nu(kr) exp(-a r^2) dr
  = k^nu exp(-k^2/4a) / (2a)^(nu+1)  with j_l(x) = sqrt(pi/2x) J_(l+1/2)(x).
* ``quadrature_sbt``: the O(N^2) midpoint-rule value of eq. BesselProj on the
  grid, sqrt(2/pi) sum_i chi_l(k_n r_i) psi(r_i) dr, with chi_l(x) = x j_l(x)
  (eq. krBessel) from SciPy.
* ``corrected_momenta``: k_nl of eq. kcorr, the j-th positive root of chi_l
  (even l) or of chi_l' (odd l) divided by rmax, j = n - n_0l + 1 (reading R9).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import spherical_jn

__all__ = ["gaussian_sbt", "chi", "chi_prime", "quadrature_sbt", "corrected_momenta"]


def gaussian_sbt(k: np.ndarray, ell: int, a: float) -> np.ndarray:
    k = np.asarray(k, dtype=np.float64)
    return k ** (ell + 1) * np.exp(-k * k / (4.0 * a)) / (2.0 * a) ** (ell + 1.5)


def chi(ell: int, x):
    """chi_l(x) = x j_l(x) (eq. krBessel)."""
    return x * spherical_jn(ell, x)


def chi_prime(ell: int, x):
    """d/dx [x j_l(x)] = j_l(x) + x j_l'(x)."""
    return spherical_jn(ell, x) + x * spherical_jn(ell, x, derivative=True)


def quadrature_sbt(psi_fn, N: int, rmax: float, ell: int, ks: np.ndarray) -> np.ndarray:
    """sqrt(2/pi) * sum_i chi_l(k r_i) psi(r_i) dr on r_i = (i - 1/2) dr."""
    dr = rmax / N
    r = (np.arange(1, N + 1) - 0.5) * dr
    f = psi_fn(r)
    return np.array([math.sqrt(2.0 / math.pi) * np.sum(chi(ell, k * r) * f) * dr for k in ks])


def corrected_momenta(N: int, rmax: float, ell: int) -> np.ndarray:
    """k_nl for the regular rows n = n_0l..N_l (eq. kcorr), in row order.

    Roots are counted from x = 0 on a fine scan and refined with Brent's method,
    so the n_0l-th row takes the first positive root (the basis function with
    the fewest nodes, Sec. 3).
    """
    p = 1 if ell % 2 == 0 else 0
    n0 = (ell + 2) // 2
    Nl = N + p - 1
    need = Nl - n0 + 1
    fn = (lambda x: chi(ell, x)) if p == 1 else (lambda x: chi_prime(ell, x))
    roots = []
    step = 0.02
    x0 = 1e-3
    f0 = fn(x0)
    xmax = (Nl + ell + 4) * math.pi
    while len(roots) < need:
        xs = np.arange(x0, min(x0 + 2000.0, xmax) + step, step)
        fs = fn(xs)
        fs[0] = f0
        s = np.nonzero(np.sign(fs[:-1]) * np.sign(fs[1:]) < 0)[0]
        for t in s:
            roots.append(brentq(fn, xs[t], xs[t + 1], xtol=1e-13, maxiter=200))
            if len(roots) == need:
                break
        x0, f0 = xs[-1], fs[-1]
        if x0 >= xmax and len(roots) < need:
            raise RuntimeError("root scan ran past the expected range")
    return np.array(roots) / rmax
