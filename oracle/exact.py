"""Exact-rational DLOP, DDLOP and Fourier-to-Bessel rows for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Everything is computed with ``fractions.Fraction`` from the defining
formulas, with no recurrence:

* P_l(i, N) = sum_j l(l, j) i^(j falling) / N^(j falling), where l(l, j) are
  the coefficients of the shifted Legendre polynomial P_l(1 - 2x)
  (Sec. 2.3, the expansion below eq. DLOPnormfac);
* the norm factor N(l, N) of eq. DLOPnormfac;
* the DDLOP P'_l(i, N) = 2/(1 + P_l(-1, N-1)) * nabla[P_l](i, N-1)
  (Sec. 2.3, eq. backDiff);
* the rows of I - L with theta(0) = 1/2 (Sec. 2.4, eq. Tdef, Ldef, step_func),
  kept as w_m * R_nm with R rational, and the completion rows of eq. Tadd.

These pin the FP64 oracle (``oracle.dsbt``) and the paper's own identities
(eq. DLOPortho, intDPx, sumDDPp, orthoImL, DLOPparity) exactly.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

__all__ = [
    "legendre_shift_coef", "falling", "dlop", "norm_factor", "ddlop",
    "imL_rows", "completion_rows", "w_sq",
]


def legendre_shift_coef(ell: int, j: int) -> int:
    """Coefficient of x^j in P_l(1 - 2x): (-1)^j C(l, j) C(l + j, j)."""
    return (-1) ** j * comb(ell, j) * comb(ell + j, j)


def falling(i: int, j: int) -> int:
    """i^(j falling) = i (i-1) ... (i-j+1); 1 for j = 0.  i may be negative."""
    out = 1
    for t in range(j):
        out *= i - t
    return out


def dlop(ell: int, i: int, N: int) -> Fraction:
    """P_l(i, N) from the falling-factorial expansion (needs l <= N)."""
    if ell > N:
        raise ValueError("degree above the number of grid intervals")
    return sum((Fraction(legendre_shift_coef(ell, j) * falling(i, j), falling(N, j))
                for j in range(ell + 1)), Fraction(0))


def norm_factor(ell: int, N: int) -> Fraction:
    """N(l, N) = (N + l + 1)^(l+1 falling) / ((2l + 1) N^(l falling)), eq. DLOPnormfac."""
    return Fraction(falling(N + ell + 1, ell + 1), (2 * ell + 1) * falling(N, ell))


def ddlop(ell: int, i: int, N: int) -> Fraction:
    """P'_l(i, N) = 2/(1 + P_l(-1, N-1)) (P_l(i, N-1) - P_l(i-1, N-1))."""
    return 2 / (1 + dlop(ell, -1, N - 1)) * (dlop(ell, i, N - 1) - dlop(ell, i - 1, N - 1))


def w_sq(m: int) -> Fraction:
    """(sqrt(1 - delta_m0/2))^2."""
    return Fraction(1, 2) if m == 0 else Fraction(1)


def imL_rows(N: int, ell: int) -> dict:
    """Regular rows of I - L as {n: {m: R_nm}} with (I - L)_nm = w_m R_nm.

    L_nm = -theta(n - m) P'_l(n - m, 2n) w_m and theta(0) = 1/2, so
    R_nm = delta_nm + theta(n - m) P'_l(n - m, 2n) (w_n = 1 for n >= 1).
    """
    p = 1 if ell % 2 == 0 else 0
    n0 = (ell + 2) // 2
    Nl = N + p - 1
    rows = {}
    for n in range(n0, Nl + 1):
        r = {}
        for m in range(p, n + 1):
            th = Fraction(1, 2) if m == n else Fraction(1)
            r[m] = (1 if m == n else 0) + th * ddlop(ell, n - m, 2 * n)
        rows[n] = r
    return rows


def completion_rows(N: int, ell: int) -> dict:
    """Completion rows of eq. Tadd without alpha and w: {n: {m: P_{l(n)}(N_l - m, 2N_l)}}."""
    p = 1 if ell % 2 == 0 else 0
    n0 = (ell + 2) // 2
    Nl = N + p - 1
    return {n: {m: dlop(2 * n - p, Nl - m, 2 * Nl) for m in range(p, Nl + 1)}
            for n in range(p, n0)}
