"""The paper's own fast Fourier-to-Bessel multiplication with monomial moments.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.6 writes the DDLOP of a regular row as a polynomial in the column
index, P'_l(n - m, 2n) = -sum_nu xi_nu(n) m^nu (eq. DP_expan), and obtains
every regular row n >= n_0 from weighted prefix sums of m^nu f_m:

    b_n = alpha_n f_n - alpha_n sum_nu xi_nu(n) s_nu,n                 (eq. fast_b_f)
    s_nu,n = delta_nu0 f_0 / sqrt(2) + sum_{m=1}^{n-1} m^nu f_m + n^nu f_n / 2
                                                                        (eq. sum_in_b_f)
    s_nu,n = s_nu,n-1 + [n^nu f_n + (n-1)^nu f_{n-1}] / 2               (eq. rec_sum_b_f)

and the inverse from suffix sums of alpha_n xi_nu(n) b_n (eqs. fast_f_b,
sum_in_f_b, fast_f_b_lowm, rec_sum_f_b).  The completion rows n < n_0 are
dense products with the rows of eq. Tadd (eq. lown_b_vs_f).

Only the coefficients with nu of the parity of l + 1 are nonzero (the DDLOP
parity), ceil(l/2) of them.  The recurrence of eq. rec_sum_b_f reproduces
eq. sum_in_b_f from n = 2 on; s_nu,1 is taken from eq. sum_in_b_f itself
(the f_0 weight 1/sqrt(2) is not of the recurrence's form).

The coefficients xi come exactly from the falling-factorial form of the DLOP
(Sec. 2.3) in rational arithmetic and are rounded to FP64 once; the sums run
in FP64 in the paper's order.  The monomial sums cancel terms far larger than
the result, so the error grows quickly with l: this module exists to measure
that and to check a GPU implementation of the same printed algorithm.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

from . import dsbt, exact

__all__ = ["xi_exact", "nonzero_nus", "tables", "forward_literal", "inverse_literal"]


def xi_exact(ell: int, n: int) -> list:
    """xi_nu(n), nu = 0..l-1, as Fractions: minus the coefficient of m^nu in
    P'_l(n - m, 2n) = 2/(1 + P_l(-1, 2n-1)) sum_j l(l, j) j (n-1-m)^(j-1 falling) / (2n-1)^(j falling)
    (the backward difference of the falling-factorial DLOP, Sec. 2.3)."""
    M = 2 * n - 1
    c = Fraction(2) / (1 + exact.dlop(ell, -1, M))
    acc = [Fraction(0)] * max(ell, 1)
    prod = [1]                      # coefficients in m of (n - 1 - m)^(j-1 falling)
    for j in range(1, ell + 1):
        if j >= 2:
            a = n - j + 1               # next factor (a - m)
            nxt = [0] * (len(prod) + 1)
            for t, v in enumerate(prod):
                nxt[t] += a * v
                nxt[t + 1] -= v
            prod = nxt
        coef = Fraction(exact.legendre_shift_coef(ell, j) * j, exact.falling(M, j))
        for t, v in enumerate(prod):
            acc[t] += coef * v
    return [-c * a for a in acc[:ell]]


def nonzero_nus(ell: int) -> list:
    return [nu for nu in range(ell) if (nu - ell - 1) % 2 == 0]


@functools.lru_cache(maxsize=32)
def tables(N: int, ell: int):
    """FP64 tables of one (N, l): {n: xi row (length l)}, {n: alpha_n} for the
    regular rows, and the dense completion rows of T (slot order)."""
    p, nz = dsbt.parity_p(ell), dsbt.n0(ell)
    Nl = dsbt.n_top(N, ell)
    T = dsbt.ftb_matrix(N, ell)
    xi, alpha = {}, {}
    for n in range(nz, Nl + 1):
        xe = xi_exact(ell, n)
        xi[n] = np.array([float(v) for v in xe])
        # (I - L)_nn = 1 + P'_l(0, 2n)/2 (theta(0) = 1/2; P'_l(0, 2n) is the
        # expansion at m = n), and T_nn = alpha_n (I - L)_nn (eq. Tdef)
        d = 1 - Fraction(1, 2) * sum(x * n ** nu for nu, x in enumerate(xe))
        alpha[n] = T[n - p, n - p] / float(d)
    return xi, alpha, T[: nz - p].copy()


def _pw(m: int, nu: int) -> float:
    return float(m) ** nu


def forward_literal(f: np.ndarray, ell: int) -> np.ndarray:
    """b = T f for one channel (f in slot order, FP64 complex) by eqs. fast_b_f,
    sum_in_b_f and rec_sum_b_f, completion rows by eq. lown_b_vs_f."""
    N = f.shape[0]
    p, nz = dsbt.parity_p(ell), dsbt.n0(ell)
    Nl = dsbt.n_top(N, ell)
    xi, alpha, C = tables(N, ell)
    nus = nonzero_nus(ell)
    fm = lambda m: f[m - p] if m >= p else 0.0
    b = np.zeros(N, dtype=np.complex128)
    b[: nz - p] = C @ f
    s = {}
    for n in range(1, Nl + 1):
        for nu in nus:
            if n == 1:
                s[nu] = (fm(0) / math.sqrt(2.0) if (nu == 0 and p == 0) else 0.0) + 0.5 * _pw(1, nu) * fm(1)
            else:
                s[nu] = s[nu] + 0.5 * (_pw(n, nu) * fm(n) + _pw(n - 1, nu) * fm(n - 1))
        if n >= nz:
            acc = 0.0
            for nu in nus:
                acc = acc + xi[n][nu] * s[nu]
            b[n - p] = alpha[n] * fm(n) - alpha[n] * acc
    return b


def inverse_literal(b: np.ndarray, ell: int) -> np.ndarray:
    """f = T^T b for one channel by eqs. fast_f_b, sum_in_f_b, fast_f_b_lowm and
    rec_sum_f_b (suffix sums from the top row down)."""
    N = b.shape[0]
    p, nz = dsbt.parity_p(ell), dsbt.n0(ell)
    Nl = dsbt.n_top(N, ell)
    xi, alpha, C = tables(N, ell)
    nus = nonzero_nus(ell)
    g = C.T @ b[: nz - p]                      # sum over completion rows n < n_0
    bn = lambda n: b[n - p]
    term = lambda n, nu: alpha[n] * xi[n][nu] * bn(n)
    f = np.zeros(N, dtype=np.complex128)
    st = {}
    for m in range(Nl, nz - 1, -1):
        for nu in nus:
            if m == Nl:
                st[nu] = 0.5 * term(m, nu)
            else:
                st[nu] = st[nu] + 0.5 * (term(m, nu) + term(m + 1, nu))
        acc = 0.0
        for nu in nus:
            acc = acc + _pw(m, nu) * st[nu]
        f[m - p] = g[m - p] + alpha[m] * bn(m) - acc
    half = {nu: st[nu] + 0.5 * term(nz, nu) for nu in nus} if nus else {}
    for m in range(p, nz):
        w = math.sqrt(0.5) if m == 0 else 1.0
        acc = 0.0
        for nu in nus:
            acc = acc + w * _pw(m, nu) * half[nu]
        f[m - p] = g[m - p] - acc
    return f
